// phase_common.h -- shared pieces of the 6D phase-space FoF kernels.
//
// Node normalisation (dispersions) uses exact integer moments, so any
// summation order -- wave shuffles, LDS atomics, global atomics -- gives the
// same result:
//   Q = rint(x * 2^20) (fp64), relative to the node's smallest-index member
//   in the nearest periodic image (integer arithmetic), W = rint(v * 2^10);
//   per axis S1 = sum(delta), S2 = sum(delta^2) (128-bit);
//   V = sum_axes (N*S2 - S1^2) = N^2 * sigma^2 in quantum units;
//   a = fl32(((double)N*(double)N / f64(V)) * 2^40), c likewise with 2^20,
//   and 1 when V = 0.
#pragma once

#include <vector>

#include "common.h"

namespace rs {

constexpr int SMALL_MAX = 2048;   // largest node handled inside one workgroup

struct PhaseParams {
    float L, h;
    int64_t LQ;        // rint(L * 2^20)
    int32_t min_sub;
    int64_t f_ppm;     // llround(f * 1e6)
    int32_t want_feat; // compute proposer features for every node
};

// node record store (slots allocated by atomics, canonical order at the end)
struct NodeRec {
    int32_t *level, *minidx, *parent, *size;
    float *l2, *a, *c, *sx2, *sv2;
    int32_t* count;     // device counter of used slots
    int32_t cap;
    int32_t* overflow;  // set when a slot beyond cap was requested
    float* feat;        // [cap * RS_NFEAT] proposer features, or NULL
};

// SoA member buffer
struct Members {
    float *x, *y, *z, *vx, *vy, *vz;
    int32_t* idx;
};

// a node whose whole subtree is split inside one workgroup
struct SmallItem {
    int32_t slot, level, size, refidx;   // refidx: smallest member particle index
    int64_t off;                         // first member in its member buffer
};

// a large node handed to the next level of the large-node pipeline
struct ChildOut {
    int32_t slot, size, minidx, level;
    int64_t off;                         // first member in its member buffer
};

struct LNode {              // one large node of the current level
    int32_t slot, size, minidx, level;
    int64_t in_off;         // first member in the input buffer
    int64_t t_off;          // first member in tile order
    int32_t tile0, ntile, super0, nsuper;
    int32_t item0, nitem;   // first (node, chunk) work item, and their count
};

struct LItem {              // (node, chunk) work item
    int32_t v, len;
    int64_t in_start, t_start;
};

// a rejected bracket is refined in up to two steps.  Below lo: the queries
// within lo are searched again with a stop at their first neighbour within
// a lower threshold (REFINE_LO2 lo^2), exactly only when the k-th value lies
// below it.  Above hi: the queries beyond hi are searched capped at
// REFINE_CAP2 hi^2, without a cap only when the k-th value lies beyond it.
constexpr float REFINE_LO2 = 0.81f;    // (0.9)^2
constexpr float REFINE_CAP2 = 1.21f;   // (1.1)^2

struct LParam {
    float a, c, sa, sc;
    float rx, ry, rz;       // reference member position
    float cx, cy, cz;       // mean position (sort key and feature centre)
    float cu, cv, cw;       // mean velocity (sort key and feature centre)
    int32_t nowrap, cull;
    uint32_t pf, pm;        // radix-select prefix and mask
    int32_t kk;             // remaining rank
    float l2;
    int32_t nnmode;         // 0 exact, 1 bracket, 2 done, 3/4 refine below lo / above hi,
                            // 6/5 the second refinement step below / above
    float lo2, hi2;         // bracket (squares) when nnmode == 1
    float isx, isv;         // 1/sigma_x, 1/sigma_v for the feature histograms
};

struct LCounters {
    int32_t n_small, n_large;
    unsigned long long tot_small, tot_large;
};

// search tree over the members of the large nodes of one level
struct TreeBuf {
    int32_t *istart, *iend, *ientry, *cfirst, *ccount;   // internal nodes [cap_inode]
    int32_t *estart, *eend, *enode;                       // child entries [cap_entry]
    float* erec;   // [16 * cap_entry]: lo xyz uvw, hi xyz uvw, then (int) start end cfirst ccount
    int32_t* leaf_of;                                     // [members] leaf entry of each member
    int32_t *n_inode, *n_entry, *overflow;                // device counters
    int32_t cap_inode, cap_entry;
};

struct TArgs {
    const int32_t* mnode;    // [members] node of each member (tile order)
    const int32_t* tile_node;
    const LNode* nodes;
    const LParam* prm;
    const int32_t* root;     // [node] root internal node
    TreeBuf tb;
    Members T;
    PhaseParams pp;
    int64_t nmem;            // members at this level
};

// Absolute slack of the box lower bounds on unwrapped positions: it covers
// the fp32 rounding of each member's position relative to the node's
// reference member, of the pair difference and of the image shift (at most
// 3 units of 2^-24 L) and the rounding of the bound's own differences.  The
// search tree stores its position boxes widened by it (rounded outward), so
// that a bound is the plain gap to the widened box.
__host__ __device__ inline float box_slack(float L) { return 8.0f * L * 5.9604645e-08f; }

// A member's coordinate.  With O32 (fewer than 2^30 members) the byte offset
// is formed in 32 bits, so the six loads of one member share one offset
// register and address from the uniform array bases.
template <bool O32>
RS_DEV float mload(const float* __restrict__ base, int64_t m) {
    if constexpr (O32)
        return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) +
                                               ((uint32_t)m << 2));
    else
        return base[m];
}
constexpr int64_t O32_LIMIT = (int64_t)1 << 30;
// 32-bit member offsets below O32_LIMIT members; the test hook
// RS_DEBUG_WIDE_OFFSETS selects the 64-bit form on any level
bool use_o32(int64_t nmem);

int tree_build(TreeBuf& tb, int32_t* root, const uint64_t* skeys, const LNode* nodes, int nv,
               const Members& T, const int32_t* mnode, const LParam* prm,
               const PhaseParams& pp, std::vector<int32_t>* level_begin, bool* overflow,
               int32_t* n_entry_out, hipStream_t st);
// refits the leaf and internal boxes to the members with d_i^2 <= l^2 (after
// the select, before linking)
int tree_refit_active(TreeBuf& tb, int32_t n_entry, const std::vector<int32_t>& level_begin,
                      const Members& T, const int32_t* mnode, const LParam* prm,
                      const PhaseParams& pp, const float* d2, hipStream_t st);
// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Blocks are remapped so that every XCD runs consecutive chunks of C
// tiles: neighbouring tiles, which read mostly the same candidate data, then
// share one L2.  The grid is rounded up to whole rounds of 8*C blocks; the
// mapping is a bijection on the rounded range, and blocks whose tile index
// is past the end exit.
constexpr int XCDS = 8;
RS_DEV int xcd_chunk_index(int b, int C) {
    const int x = b % XCDS, r = b / XCDS;
    return ((r / C) * XCDS + x) * C + r % C;
}
inline int xcd_chunk_grid(int n, int C) {
    const int g = XCDS * C;
    return (n + g - 1) / g * g;
}
// chunk length: whole rounds stay at least 64 so the XCDs finish together;
// the longest chunk comes from the tuning table
inline int xcd_chunk(int ntiles) {
    const int cap = tune_get(TUNE_XCD_CHUNK);
    int c = ntiles / (64 * XCDS);
    return c < 1 ? 1 : (c > cap ? cap : c);
}

int tree_nn(const TArgs& A, int ntiles, float* d2, hipStream_t st);
int tile_link(const TArgs& A, int ntiles, const float* d2, int32_t* par, hipStream_t st);


// device buffers of the large-node pipeline, sized by the level-0 total of
// large-node members (which bounds every later level)
struct LargeWork {
    int64_t cap_m, cap_nodes, cap_items, cap_tiles, cap_supers, cap_small;
    Members T;           // this level's members in 6D Morton order
    Members SN;          // children: small ones from the front, large ones from the back
    uint64_t *kin, *kout;
    int32_t *src, *perm, *mnode, *par, *cnt, *cslot, *cfill;
    int64_t* coff;
    int8_t* cclass;
    unsigned long long* mpk;
    float* d2;
    float* lrec;   // interleaved member records of the level's gather (aliases par..d2)
    LNode* nodes;
    LItem* items;
    LParam* prm;
    unsigned long long* gacc;
    uint32_t* gext;
    int32_t* ghist;
    int32_t *tile_node, *super_node;
    float *tbox, *sbox;
    LCounters* ctr;
    SmallItem* small_items;
    SmallItem* buckets;
    int32_t* bcount;
    ChildOut* large_out;
    void* sort_temp;
    size_t sort_temp_bytes;
    TreeBuf tb;
    int32_t* root;
    int32_t* lhist;      // [16 * cap_nodes] feature histograms
    float* lfeat;        // [RS_NFEAT * cap_nodes] features of the level's large nodes
    float* lnl;          // [cap_nodes] proposed ln(l)
    int32_t* lcnt;       // [2 * cap_nodes] bracket counts #(<= lo), #(<= hi)
    int32_t* lstat;      // [4] accepted, fell back
    const float* model;  // device copy of the proposer, or NULL (exact search)
    // small children of a level run on `side` (when set) while the next level
    // proceeds; side_done marks their end, side_pending that one is in flight
    hipStream_t side = nullptr;
    hipEvent_t side_ready = nullptr, side_done = nullptr;
    bool side_pending = false;
};

size_t large_work_bytes(int64_t m, int32_t min_sub);
int large_work_carve(Arena* ar, int64_t m, int32_t min_sub, LargeWork* w);
// (re)reserves the search-tree buffers for up to m members and nv nodes;
// grow > 1 multiplies the entry and internal-node capacities
int tree_reserve(LargeWork* w, int64_t m, int64_t nv, int64_t grow);
int launch_small_items(LargeWork* w, const SmallItem* items, int n, const Members& mb,
                       const NodeRec& nr, const PhaseParams& pp, int32_t* deepest,
                       hipStream_t st);
int large_level(LargeWork* w, const std::vector<ChildOut>& hn, const Members& in,
                const float* X, const float* Y, const float* Z, const PhaseParams& pp,
                const NodeRec& nr, int32_t* deepest, std::vector<ChildOut>* next,
                int64_t* n_accepted, int64_t* n_fallback, hipStream_t st);
int mlp_infer(const float* model_dev, int nv, const float* feat, float* out, hipStream_t st);
int run_small_bucket(int b, const SmallItem* items, int n_items, const Members& mb,
                     const NodeRec& nr, const PhaseParams& pp, int32_t* deepest,
                     hipStream_t st,
                     const char* timer = "phase_small");
int small_bucket_of(int size);

RS_DEV int64_t select_rank(int64_t n, int64_t ppm) {
    int64_t k = (n * ppm + 999999) / 1000000;
    return k < 1 ? 1 : (k > n ? n : k);
}

RS_DEV int64_t quant_pos(float x) { return (int64_t)rint((double)x * 1048576.0); }
RS_DEV int64_t quant_vel(float v) { return (int64_t)rint((double)v * 1024.0); }

// 18 words: s1[0..5] (pos xyz, vel xyz; two's complement), then s2 lo/hi
// pairs for the same six quantities.
struct Moments {
    uint64_t s1[6];
    u128 s2[6];
};

RS_DEV void mom_zero(Moments& m) {
#pragma unroll
    for (int q = 0; q < 6; q++) {
        m.s1[q] = 0;
        m.s2[q] = 0;
    }
}

RS_DEV void mom_add(Moments& m, float px, float py, float pz, float vx, float vy, float vz,
                    const int64_t qref[3], int64_t LQ) {
    float p[3] = {px, py, pz};
    float v[3] = {vx, vy, vz};
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
        int64_t d = quant_pos(p[ax]) - qref[ax];
        if (2 * d > LQ) d -= LQ;
        else if (2 * d <= -LQ) d += LQ;
        m.s1[ax] += (uint64_t)d;
        m.s2[ax] += (u128)(uint64_t)(d * d);
        int64_t w = quant_vel(v[ax]);
        m.s1[3 + ax] += (uint64_t)w;
        m.s2[3 + ax] += (u128)(uint64_t)(w * w);
    }
}

RS_DEV uint64_t shfl_xor_u64(uint64_t v, int mask) {
    uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, mask, 64);
    uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), mask, 64);
    return ((uint64_t)hi << 32) | lo;
}

// sum over the 64 lanes (every lane ends with the total)
RS_DEV void mom_wave_reduce(Moments& m) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int q = 0; q < 6; q++) {
            m.s1[q] += shfl_xor_u64(m.s1[q], off);
            uint64_t lo = (uint64_t)m.s2[q], hi = (uint64_t)(m.s2[q] >> 64);
            uint64_t olo = shfl_xor_u64(lo, off), ohi = shfl_xor_u64(hi, off);
            m.s2[q] += ((u128)ohi << 64) | (u128)olo;
        }
    }
}

// add one wave's moments into an 18-word accumulator (LDS or global)
RS_DEV void acc_add128(unsigned long long* lo_p, unsigned long long* hi_p, u128 v) {
    unsigned long long lo = (unsigned long long)(uint64_t)v;
    unsigned long long hi = (unsigned long long)(uint64_t)(v >> 64);
    unsigned long long old = atomicAdd(lo_p, lo);
    unsigned long long carry = (old + lo) < old ? 1ull : 0ull;
    atomicAdd(hi_p, hi + carry);
}

RS_DEV void mom_accumulate(unsigned long long* acc, const Moments& m) {
#pragma unroll
    for (int q = 0; q < 6; q++) atomicAdd(acc + q, (unsigned long long)m.s1[q]);
#pragma unroll
    for (int q = 0; q < 6; q++) acc_add128(acc + 6 + 2 * q, acc + 7 + 2 * q, m.s2[q]);
}

struct Norm {
    float a, c, sx2, sv2;
    double mean[6];   // mean position offset (from ref, fp64) and mean velocity
};

RS_DEV Norm mom_finalize(const unsigned long long* acc, int64_t n) {
    i128 Vx = 0, Vv = 0;
    Norm r;
#pragma unroll
    for (int q = 0; q < 6; q++) {
        int64_t s1 = (int64_t)acc[q];
        u128 s2 = ((u128)acc[7 + 2 * q] << 64) | (u128)acc[6 + 2 * q];
        i128 t = (i128)n * (i128)s2 - (i128)s1 * (i128)s1;
        if (q < 3) Vx += t; else Vv += t;
        r.mean[q] = (double)s1 / (double)n * (q < 3 ? 9.5367431640625e-07 : 9.765625e-4);
    }
    double nn = (double)n * (double)n;
    double vx = i128_to_f64(Vx), vv = i128_to_f64(Vv);
    r.a = (Vx == 0) ? 1.0f : (float)((nn / vx) * 1099511627776.0);
    r.c = (Vv == 0) ? 1.0f : (float)((nn / vv) * 1048576.0);
    r.sx2 = (float)((vx / nn) * 9.094947017729282e-13);
    r.sv2 = (float)((vv / nn) * 9.5367431640625e-07);
    return r;
}

// pair metric for one candidate, with or without the periodic shift
template <bool WRAP>
RS_DEV float phase_d2(float xi, float yi, float zi, float ui, float vi, float wi, float xj,
                      float yj, float zj, float uj, float vj, float wj, float a, float c,
                      float L, float h) {
    float Dx = WRAP ? pos_d2_wrap(xi, yi, zi, xj, yj, zj, L, h)
                    : pos_d2_nowrap(xi, yi, zi, xj, yj, zj);
    float Dv = sum_sq3(ui - uj, vi - vj, wi - wj);
    return metric(a, Dx, c, Dv);
}

// ---------------------------------------------------------------------------
// proposer features (see RS_NFEAT in rsfof.h)
// ---------------------------------------------------------------------------

RS_DEV int feat_bin(float t) {
    return (t >= 0.25f) + (t >= 0.5f) + (t >= 0.75f) + (t >= 1.0f) + (t >= 1.5f) + (t >= 2.0f) +
           (t >= 3.0f);
}

// centre and scale used for the histograms of one node
struct FeatFrame {
    float cx, cy, cz, cu, cv, cw;   // mean position (may lie outside the box) and velocity
    float isx, isv;                 // 1/sigma (0 when sigma = 0)
};

RS_DEV FeatFrame feat_frame(const unsigned long long* acc, int64_t n, float rx, float ry,
                            float rz, float sx2, float sv2) {
    FeatFrame f;
    double m[6];
    for (int q = 0; q < 6; q++)
        m[q] = (double)(int64_t)acc[q] / (double)n * (q < 3 ? 9.5367431640625e-07 : 9.765625e-4);
    f.cx = (float)((double)rx + m[0]);
    f.cy = (float)((double)ry + m[1]);
    f.cz = (float)((double)rz + m[2]);
    f.cu = (float)m[3];
    f.cv = (float)m[4];
    f.cw = (float)m[5];
    f.isx = sx2 > 0.0f ? 1.0f / sqrtf(sx2) : 0.0f;
    f.isv = sv2 > 0.0f ? 1.0f / sqrtf(sv2) : 0.0f;
    return f;
}

RS_DEV void feat_member_bins(const FeatFrame& f, float x, float y, float z, float u, float v,
                             float w, float L, float h, int* br, int* bv) {
    float r2 = sum_sq3(min_image(x - f.cx, L, h), min_image(y - f.cy, L, h),
                       min_image(z - f.cz, L, h));
    float v2 = sum_sq3(u - f.cu, v - f.cv, w - f.cw);
    *br = feat_bin(sqrtf(r2) * f.isx);
    *bv = 8 + feat_bin(sqrtf(v2) * f.isv);
}

RS_DEV void feat_write(float* out, const unsigned long long* acc, int64_t n, int level,
                       const int32_t* hist16) {
    i128 t[6], Vx = 0, Vv = 0;
    for (int q = 0; q < 6; q++) {
        int64_t s1 = (int64_t)acc[q];
        u128 s2 = ((u128)acc[7 + 2 * q] << 64) | (u128)acc[6 + 2 * q];
        t[q] = (i128)n * (i128)s2 - (i128)s1 * (i128)s1;
        if (q < 3) Vx += t[q]; else Vv += t[q];
    }
    out[0] = logf((float)n);
    for (int q = 0; q < 3; q++) {
        out[1 + q] = Vx > 0 ? (float)(i128_to_f64(t[q]) / i128_to_f64(Vx)) : (1.0f / 3.0f);
        out[4 + q] = Vv > 0 ? (float)(i128_to_f64(t[3 + q]) / i128_to_f64(Vv)) : (1.0f / 3.0f);
    }
    for (int b = 0; b < 16; b++) out[7 + b] = (float)hist16[b] / (float)n;
    out[23] = (float)level;
}

// lock-free union-find in LDS (same invariant as the global version)
RS_DEV int lds_find(int* par, int v) {
    int cur = __hip_atomic_load(par + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (cur == v) return v;
    int prev = v, next;
    while (cur > (next = __hip_atomic_load(par + cur, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP))) {
        __hip_atomic_store(par + prev, next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        prev = cur;
        cur = next;
    }
    return cur;
}

// read-only root walk, for flattening: stores nothing but the final root, so
// concurrent flatteners never overwrite a root entry with an older ancestor
RS_DEV int lds_root(const int* par, int v) {
    int cur = __hip_atomic_load(par + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (cur != v) {
        v = cur;
        cur = __hip_atomic_load(par + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    return v;
}

RS_DEV void lds_unite(int* par, int a, int b) {
    int ra = lds_find(par, a), rb = lds_find(par, b);
    while (ra != rb) {
        if (ra > rb) { int t = ra; ra = rb; rb = t; }
        int old = atomicCAS(par + rb, rb, ra);
        if (old == rb) return;
        rb = lds_find(par, old);
        ra = lds_find(par, ra);
    }
}

}  // namespace rs
