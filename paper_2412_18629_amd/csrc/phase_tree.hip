// phase_tree.hip -- 6D search tree over the Morton-sorted members of the
// large nodes of one level, and the nearest-neighbour / linking traversals.
//
// Tree: an internal node is a Morton-prefix cell (6 key bits per level, one
// per dimension) with more than 64 members.  Its children are the non-empty
// sub-cells of the next level: sub-cells with more than 64 members become
// internal nodes, runs of consecutive smaller sub-cells are packed into
// leaves of at most 64 members.  Cells of the finest level are cut into
// 64-member leaves.  Every child entry carries the exact bounding box of its
// members (positions unwrapped around the node's reference member, raw
// velocities), so boxes are tight at every level.
//
// Traversal: one wavefront handles one query at a time.  The 64 lanes bound
// 64 child boxes in parallel (two cells of at most 32 children share a
// pass); surviving leaves are scanned one candidate per lane, surviving
// internal children go onto a per-wavefront LDS stack, the nearest on top.
#include "phase_common.h"

namespace rs {

constexpr uint64_t MORTON_MASK = (1ull << 42) - 1ull;
constexpr int TREE_LEVELS = 7;       // 42 Morton bits, 6 per level
constexpr int STACK_PER_WAVE = 520;  // >= 64 internal children x 8 levels

// first position in [lo, hi) whose Morton bits are >= target
RS_DEV int32_t morton_lower_bound(const uint64_t* __restrict__ keys, int32_t lo, int32_t hi,
                                  uint64_t target) {
    while (lo < hi) {
        int32_t mid = lo + ((hi - lo) >> 1);
        if ((keys[mid] & MORTON_MASK) < target) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// One wavefront per internal node of `level`, four per block: find its
// children by lane-parallel binary search (lane d -> digit d), pack the
// small ones into leaves, allocate entries and child internal nodes.  The
// inode and entry counters are adjacent, so one 64-bit atomic per block
// reserves both for its four nodes (one counter hit by every node was the
// cost of this kernel).
constexpr int SPLIT_WAVES = 4;

__global__ void __launch_bounds__(64 * SPLIT_WAVES)
k_tree_split(const uint64_t* __restrict__ keys, int32_t node_begin, int32_t node_end, int level,
             TreeBuf tb) {
    __shared__ unsigned long long req[SPLIT_WAVES];
    __shared__ unsigned long long sbase;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int32_t x = node_begin + blockIdx.x * SPLIT_WAVES + w;
    const bool valid = x < node_end;
    const int32_t start = valid ? tb.istart[x] : 0, end = valid ? tb.iend[x] : 0;
    const int32_t cnt_all = end - start;
    const bool finest = level >= TREE_LEVELS;
    int32_t n_int = 0, n_ent = 0, lo = 0, cnt = 0;
    if (finest) {
        // finest cell: cut into 64-member leaves
        n_ent = (cnt_all + 63) / 64;
    } else if (valid) {
        const int shift = 42 - 6 * (level + 1);
        const uint64_t prefix = (keys[start] & MORTON_MASK) >> (shift + 6);
        const uint64_t target = ((prefix << 6) | (uint64_t)lane) << shift;
        lo = morton_lower_bound(keys, start, end, target);
        int32_t hi = __shfl_down(lo, 1, 64);
        if (lane == 63) hi = end;
        cnt = hi - lo;
        // every lane runs the packing walk over the 64 digits (values
        // broadcast by shuffles), so all counts agree
        int32_t run = 0;
        for (int d = 0; d < 64; d++) {
            const int32_t c = __shfl(cnt, d, 64);
            if (c == 0) continue;
            if (c > 64) {
                if (run) { n_ent++; run = 0; }
                n_int++;
                n_ent++;
            } else if (run + c > 64) {
                n_ent++;
                run = c;
            } else {
                run += c;
            }
        }
        if (run) n_ent++;
    }
    if (lane == 0) req[w] = ((unsigned long long)n_ent << 32) | (unsigned long long)n_int;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int k = 0; k < SPLIT_WAVES; k++) tot += req[k];
        // low word: n_inode, high word: n_entry
        sbase = atomicAdd(reinterpret_cast<unsigned long long*>(tb.n_inode), tot);
    }
    __syncthreads();
    if (!valid) return;
    unsigned long long bw = sbase;
    for (int k = 0; k < w; k++) bw += req[k];
    const int32_t ibase = (int32_t)(bw & 0xffffffffull), ebase = (int32_t)(bw >> 32);
    const bool ok = ebase + n_ent <= tb.cap_entry && ibase + n_int <= tb.cap_inode;
    if (lane == 0) {
        if (!ok) atomicOr(tb.overflow, 1);
        tb.cfirst[x] = ok ? ebase : 0;
        tb.ccount[x] = ok ? n_ent : 0;
    }
    if (!ok) return;
    if (finest) {
        for (int32_t k = lane; k < n_ent; k += 64) {
            const int32_t e = ebase + k;
            tb.estart[e] = start + 64 * k;
            tb.eend[e] = min(start + 64 * (k + 1), end);
            tb.enode[e] = -1;
        }
        return;
    }
    int32_t e = ebase, in = ibase, rs0 = -1, re0 = -1, run = 0;
    for (int d = 0; d < 64; d++) {
        const int32_t c = __shfl(cnt, d, 64);
        const int32_t l0 = __shfl(lo, d, 64);
        if (c == 0) continue;
        if (c > 64) {
            if (run) {
                if (lane == 0) { tb.estart[e] = rs0; tb.eend[e] = re0; tb.enode[e] = -1; }
                e++;
                run = 0;
            }
            if (lane == 0) {
                tb.estart[e] = l0; tb.eend[e] = l0 + c; tb.enode[e] = in;
                tb.istart[in] = l0; tb.iend[in] = l0 + c; tb.ientry[in] = e;
            }
            in++;
            e++;
        } else if (run + c > 64) {
            if (lane == 0) { tb.estart[e] = rs0; tb.eend[e] = re0; tb.enode[e] = -1; }
            e++;
            rs0 = l0; re0 = l0 + c; run = c;
        } else {
            if (!run) rs0 = l0;
            re0 = l0 + c;
            run += c;
        }
    }
    if (run && lane == 0) { tb.estart[e] = rs0; tb.eend[e] = re0; tb.enode[e] = -1; }
}

RS_DEV float wmin(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

RS_DEV float wmax(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// minimum over the 64 lanes of a non-negative float (or +inf), returned
// uniform; non-negative float bit patterns order like their values.  Row
// steps (quad permutes, row rotations) leave each 16-lane row's minimum in
// all its lanes; two row broadcasts carry it to lane 63.  All 64 lanes must
// be active.  Rows a broadcast skips read the identity (all ones), so each
// step compiles to one DPP minimum instead of two moves and a minimum.
RS_DEV float wmin_nonneg(float x) {
    uint32_t v = __float_as_uint(x);
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0xB1, 0xf, 0xf, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x4E, 0xf, 0xf, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x124, 0xf, 0xf, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x128, 0xf, 0xf, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x142, 0xa, 0xf, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x143, 0xc, 0xf, false));
    return __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)v, 63));
}

// leaf boxes (wave per entry) and the leaf of every member; position
// extents widened by the bounds' slack
__global__ void __launch_bounds__(256)
k_tree_leafbox(int32_t n_entry, TreeBuf tb, Members T, const int32_t* __restrict__ mnode,
               const LParam* __restrict__ prm, PhaseParams pp) {
    const int lane = threadIdx.x & 63;
    const int32_t e = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= n_entry || tb.enode[e] >= 0) return;
    const int32_t s = tb.estart[e], t = tb.eend[e];
    const int32_t m = s + lane;
    const bool ok = m < t;
    float c[6] = {0, 0, 0, 0, 0, 0};
    if (ok) {
        const LParam P = prm[mnode[m]];
        c[0] = min_image(T.x[m] - P.rx, pp.L, pp.h);
        c[1] = min_image(T.y[m] - P.ry, pp.L, pp.h);
        c[2] = min_image(T.z[m] - P.rz, pp.L, pp.h);
        c[3] = T.vx[m];
        c[4] = T.vy[m];
        c[5] = T.vz[m];
        tb.leaf_of[m] = e;
    }
    const float slack = box_slack(pp.L);
#pragma unroll
    for (int d = 0; d < 6; d++) {
        float lo = wmin(ok ? c[d] : __builtin_huge_valf());
        float hi = wmax(ok ? c[d] : -__builtin_huge_valf());
        if (d < 3 && lo <= hi) {
            lo = nextafterf(lo - slack, -__builtin_huge_valf());
            hi = nextafterf(hi + slack, __builtin_huge_valf());
        }
        if (lane == 0) {
            tb.erec[16 * (int64_t)e + d] = lo;
            tb.erec[16 * (int64_t)e + 6 + d] = hi;
        }
    }
    if (lane == 0) {
        int32_t* ri = reinterpret_cast<int32_t*>(tb.erec + 16 * (int64_t)e);
        ri[12] = s;
        ri[13] = t;
        ri[14] = -1;
        ri[15] = 0;
    }
}

// leaf boxes over the members that can still link (d_i^2 <= l^2 of their
// node); a leaf without any gets an empty box (lo = +inf, hi = -inf), which
// every lower bound rejects.  Member ranges and leaf_of are unchanged.
__global__ void __launch_bounds__(256)
k_tree_leafbox_active(int32_t n_entry, TreeBuf tb, Members T, const int32_t* __restrict__ mnode,
                      const LParam* __restrict__ prm, PhaseParams pp,
                      const float* __restrict__ d2) {
    const int lane = threadIdx.x & 63;
    const int32_t e = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= n_entry || tb.enode[e] >= 0) return;
    const int32_t s = tb.estart[e], t = tb.eend[e];
    const int32_t m = s + lane;
    bool ok = m < t;
    float c[6] = {0, 0, 0, 0, 0, 0};
    if (ok) {
        const LParam P = prm[mnode[m]];
        ok = d2[m] <= P.l2;
        c[0] = min_image(T.x[m] - P.rx, pp.L, pp.h);
        c[1] = min_image(T.y[m] - P.ry, pp.L, pp.h);
        c[2] = min_image(T.z[m] - P.rz, pp.L, pp.h);
        c[3] = T.vx[m];
        c[4] = T.vy[m];
        c[5] = T.vz[m];
    }
    const float slack = box_slack(pp.L);
#pragma unroll
    for (int d = 0; d < 6; d++) {
        float lo = wmin(ok ? c[d] : __builtin_huge_valf());
        float hi = wmax(ok ? c[d] : -__builtin_huge_valf());
        if (d < 3 && lo <= hi) {
            lo = nextafterf(lo - slack, -__builtin_huge_valf());
            hi = nextafterf(hi + slack, __builtin_huge_valf());
        }
        if (lane == 0) {
            tb.erec[16 * (int64_t)e + d] = lo;
            tb.erec[16 * (int64_t)e + 6 + d] = hi;
        }
    }
}

// internal-node boxes of one level (children done before parents)
__global__ void __launch_bounds__(256)
k_tree_nodebox(int32_t node_begin, int32_t node_end, TreeBuf tb) {
    const int lane = threadIdx.x & 63;
    const int32_t x = node_begin + blockIdx.x * 4 + (threadIdx.x >> 6);
    if (x >= node_end) return;
    const int32_t f = tb.cfirst[x], n = tb.ccount[x];
    float lo[6], hi[6];
#pragma unroll
    for (int d = 0; d < 6; d++) {
        lo[d] = __builtin_huge_valf();
        hi[d] = -__builtin_huge_valf();
    }
    for (int32_t k = lane; k < n; k += 64) {
        const float* b = tb.erec + 16 * (int64_t)(f + k);
#pragma unroll
        for (int d = 0; d < 6; d++) {
            lo[d] = fminf(lo[d], b[d]);
            hi[d] = fmaxf(hi[d], b[6 + d]);
        }
    }
    const int32_t pe = tb.ientry[x];
#pragma unroll
    for (int d = 0; d < 6; d++) {
        float l = wmin(lo[d]), h = wmax(hi[d]);
        if (lane == 0 && pe >= 0) {
            tb.erec[16 * (int64_t)pe + d] = l;
            tb.erec[16 * (int64_t)pe + 6 + d] = h;
        }
    }
    if (lane == 0 && pe >= 0) {
        int32_t* ri = reinterpret_cast<int32_t*>(tb.erec + 16 * (int64_t)pe);
        ri[12] = tb.istart[x];
        ri[13] = tb.iend[x];
        ri[14] = f;
        ri[15] = n;
    }
}

// ---------------------------------------------------------------------------
// traversals
// ---------------------------------------------------------------------------

struct TQuery {
    float x, y, z, u, v, w;
    float wq[3], uq[3];
};

RS_DEV TQuery tq_load(const Members& T, int64_t m, const LParam& P, const PhaseParams& pp) {
    TQuery q;
    q.x = T.x[m]; q.y = T.y[m]; q.z = T.z[m];
    q.u = T.vx[m]; q.v = T.vy[m]; q.w = T.vz[m];
    q.wq[0] = min_image(q.x - P.rx, pp.L, pp.h);
    q.wq[1] = min_image(q.y - P.ry, pp.L, pp.h);
    q.wq[2] = min_image(q.z - P.rz, pp.L, pp.h);
    q.uq[0] = q.u; q.uq[1] = q.v; q.uq[2] = q.w;
    return q;
}

template <bool O32>
RS_DEV float tq_d2(const Members& T, int64_t m, const TQuery& q, const LParam& P,
                   const PhaseParams& pp) {
    const float xj = mload<O32>(T.x, m), yj = mload<O32>(T.y, m), zj = mload<O32>(T.z, m);
    const float uj = mload<O32>(T.vx, m), vj = mload<O32>(T.vy, m), wj = mload<O32>(T.vz, m);
    return P.nowrap ? phase_d2<false>(q.x, q.y, q.z, q.u, q.v, q.w, xj, yj, zj, uj, vj, wj, P.a,
                                      P.c, pp.L, pp.h)
                    : phase_d2<true>(q.x, q.y, q.z, q.u, q.v, q.w, xj, yj, zj, uj, vj, wj, P.a,
                                     P.c, pp.L, pp.h);
}

// one child-entry record, read with four 16-byte loads
struct Rec {
    float lo[6], hi[6];
    int32_t start, end, cfirst, ccount;   // cfirst < 0: leaf
};

RS_DEV Rec rec_load(const float* __restrict__ erec, int32_t k) {
    const float4* p = reinterpret_cast<const float4*>(erec + 16 * (int64_t)k);
    float4 a = p[0], b = p[1], c = p[2], d = p[3];
    Rec r;
    r.lo[0] = a.x; r.lo[1] = a.y; r.lo[2] = a.z; r.lo[3] = a.w; r.lo[4] = b.x; r.lo[5] = b.y;
    r.hi[0] = b.z; r.hi[1] = b.w; r.hi[2] = c.x; r.hi[3] = c.y; r.hi[4] = c.z; r.hi[5] = c.w;
    r.start = __float_as_int(d.x);
    r.end = __float_as_int(d.y);
    r.cfirst = __float_as_int(d.z);
    r.ccount = __float_as_int(d.w);
    return r;
}

// exact lower bound of the computed d^2 from the query to any member of a
// record's box: the position gap is to the box widened by the slack (which
// covers the rounding of x - x_ref, of the pair difference and of the image
// shift); velocity gaps and the bound itself lose a relative margin
RS_DEV float rec_lb(const Rec& r, const TQuery& q, float a, float c) {
    float sp = 0.0f, sv = 0.0f;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const float g = fmaxf(fmaxf(r.lo[d] - q.wq[d], q.wq[d] - r.hi[d]), 0.0f);
        sp += g * g;
        float h = fmaxf(fmaxf(r.lo[3 + d] - q.uq[d], q.uq[d] - r.hi[3 + d]), 0.0f) * 0.99999905f;
        sv += h * h;
    }
    return (a * sp + c * sv) * 0.99999f;
}

struct StackEnt {
    int32_t cfirst, ccount;
    float lb;
};

// A stack entry in LDS takes 8 bytes, so that eight wavefronts fit per SIMD
// (the search is bound by the latency of its dependent loads).  The child
// count (1..64) sits in the low six bits of the lower bound, whose value is
// truncated there: truncating a non-negative float only lowers it, so the
// stored bound still prunes nothing that the exact one would keep.  A finest
// cell can have more than 64 children (leaves of members that share the full
// Morton prefix); it is stored as the negated entry index of the cell, and
// its child range is read back from the cell's record when it is popped.
struct StackSlot {
    int32_t cfirst;
    uint32_t pk;
};

RS_DEV StackSlot stack_pack(int32_t entry, int32_t cfirst, int32_t ccount, float lb) {
    const uint32_t b = __float_as_uint(lb) & ~63u;
    if (ccount <= 64) return StackSlot{cfirst, b | (uint32_t)(ccount - 1)};
    return StackSlot{-1 - entry, b};
}

RS_DEV StackEnt stack_unpack(StackSlot s) {
    return StackEnt{s.cfirst, (int32_t)(s.pk & 63u) + 1, __uint_as_float(s.pk & ~63u)};
}

// nearest-neighbour d^2 of every member (exact): own leaf first, then a
// depth-first descent from the node's root.  One wavefront per tile of
// queries, one query at a time; child records are bounded lane-parallel,
// surviving leaves are scanned four at a time with independent loads.
// pair tests of the counting build (instrumentation level 2), spread over 64
// counters to keep the atomics apart
__device__ unsigned long long g_nn_pairs[64];

template <bool O32, bool CNT>
__global__ void __launch_bounds__(64)
k_tree_nn(TArgs A, int ntiles, int chunk, float* __restrict__ d2out) {
    __shared__ StackSlot stk[STACK_PER_WAVE];
    const int lane = threadIdx.x;
    const int t = xcd_chunk_index(blockIdx.x, chunk);
    if (t >= ntiles) return;
    const int v = A.tile_node[t];
    const LNode nd = A.nodes[v];
    const LParam P = A.prm[v];
    const Members& T = A.T;
    const TreeBuf& tb = A.tb;
    const int64_t ts = nd.t_off + 64ll * (t - nd.tile0);
    const int64_t te = min(ts + 64, nd.t_off + (int64_t)nd.size);
    const bool cull = P.cull != 0;
    if (P.nnmode == 2) return;               // bracket already accepted
    // bracket mode (1): searches are capped at hi^2 and stop at the first
    // neighbour within lo^2; the output encodes 0 = within lo, the exact d^2
    // in (lo^2, hi^2], +inf = nothing within hi.
    // Refinement after a rejected bracket searches only the queries that can
    // hold the k-th smallest d^2; every other stored value already orders
    // correctly against it.  Below lo^2: mode 3 searches the queries coded 0
    // (capped just above lo^2) with a stop at the first neighbour within
    // lo3 = REFINE_LO2 lo^2, coding 0 again there and the exact d^2 above;
    // mode 6, when the k-th value lies within lo3 too, searches the queries
    // still coded 0 exactly, capped just above lo3.  Above hi^2: mode 4
    // searches the queries coded +inf capped at cap4 = REFINE_CAP2 hi^2
    // (+inf beyond it); mode 5, when the k-th value lies beyond cap4 too,
    // searches the queries still coded +inf without a cap.
    const int mode = P.nnmode;
    const bool brk = mode == 1;
    const float cap4 = REFINE_CAP2 * P.hi2;
    const float lo3 = REFINE_LO2 * P.lo2;
    auto above = [](float v) { return __uint_as_float(__float_as_uint(v) + 1u); };
    const float cap = brk ? above(P.hi2)
                    : mode == 3 ? above(P.lo2)
                    : mode == 4 ? above(cap4)
                    : mode == 6 ? above(lo3)
                                : __builtin_huge_valf();
    // early stop: the first neighbour within this d^2 ends a query
    const float lo2 = brk ? P.lo2 : mode == 3 ? lo3 : -1.0f;
    const float redo = mode == 3 || mode == 6 ? 0.0f : __builtin_huge_valf();
    const bool refine = mode >= 3;
    const int32_t rf = tb.cfirst[A.root[v]], rn = tb.ccount[A.root[v]];
    unsigned long long npairs = 0;   // counting build only
    for (int64_t qm = ts; qm < te; qm++) {
        if (refine && !(d2out[qm] == redo)) continue;
        const TQuery q = tq_load(T, qm, P, A.pp);
        const int32_t e0 = tb.leaf_of[qm];
        const int32_t* r0 = reinterpret_cast<const int32_t*>(tb.erec + 16 * (int64_t)e0);
        float bl = cap;
        {
            const int64_t m = r0[12] + lane;
            if (m < r0[13] && m != qm) bl = fminf(bl, tq_d2<O32>(T, m, q, P, A.pp));
        }
        float best = wmin_nonneg(bl);
        if (CNT) npairs += (unsigned long long)(r0[13] - r0[12] - 1);
        // a node's root is never a finest cell: at most 64 children
        if (lane == 0) stk[0] = stack_pack(0, rf, rn, 0.0f);
        int sp = best <= lo2 ? 0 : 1;
        __syncthreads();
        while (sp > 0) {
            sp--;
            StackEnt se = stack_unpack(stk[sp]);
            if (se.cfirst < 0) {
                // finest cell with more than 64 leaves: its range from its record
                const float* rec = tb.erec + 16 * (int64_t)(-1 - se.cfirst);
                const int2 cc = *reinterpret_cast<const int2*>(rec + 14);
                se.cfirst = cc.x;
                se.ccount = cc.y;
            }
            // most cells have at most 32 children: the next entry, when it is
            // as small and still needed, is visited in the same pass on the
            // upper half of the lanes (the live entries of each depth still
            // come from one pass, at most 64, so the stack bound holds)
            StackEnt se2{0, 0, 0.0f};
            if (se.ccount <= 32 && sp > 0) {
                const StackEnt t2 = stack_unpack(stk[sp - 1]);
                if (t2.cfirst >= 0 && t2.ccount <= 32 && (!cull || t2.lb < best)) {
                    se2 = t2;
                    sp--;
                }
            }
            __syncthreads();
            const bool pair = se2.ccount > 0;
            if (cull && !(se.lb < best)) {
                if (!pair) continue;
                se.ccount = 0;
            }
            for (int32_t b0 = 0; b0 < se.ccount || (pair && b0 == 0); b0 += 64) {
                const bool hi_half = pair && lane >= 32;
                const int32_t k = hi_half ? se2.cfirst + lane - 32 : se.cfirst + b0 + lane;
                const bool valid = hi_half ? lane - 32 < se2.ccount
                                           : b0 + lane < se.ccount && (!pair || lane < 32);
                Rec r;
                bool need = false;
                float lb = 0.0f;
                if (valid && k != e0) {
                    r = rec_load(tb.erec, k);
                    lb = cull ? rec_lb(r, q, P.a, P.c) : 0.0f;
                    need = lb < best;
                } else {
                    r.start = r.end = 0;
                    r.cfirst = -1;
                    r.ccount = 0;
                }
                const bool leaf = r.cfirst < 0;
                const uint64_t imask = __ballot(need && !leaf);
                if (need && !leaf)
                    stk[sp + __popcll(imask & lanemask_lt())] =
                        stack_pack(k, r.cfirst, r.ccount, lb);
                if (cull && __popcll(imask) > 1) {
                    // the nearest internal child goes on top: visited first,
                    // it lowers `best` soonest and prunes its siblings
                    const float m = wmin_nonneg(need && !leaf ? lb : __builtin_huge_valf());
                    const uint64_t w = __ballot(need && !leaf && lb == m);
                    if (lane == __ffsll((unsigned long long)w) - 1) {
                        const int pos = sp + __popcll(imask & lanemask_lt());
                        const int top = sp + __popcll(imask) - 1;
                        if (pos != top) {
                            const StackSlot e = stk[top];
                            stk[top] = stk[pos];
                            stk[pos] = e;
                        }
                    }
                }
                sp += __popcll(imask);
                __syncthreads();
                uint64_t mk = __ballot(need && leaf);
                while (mk) {
                    // up to four leaves: every lane loads one member of each
                    // (a valid member where the leaf is shorter, masked
                    // afterwards), all loads before any arithmetic so that
                    // they are in flight together
                    int32_t s4[4], e4[4];
                    int cnt = 0;
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        s4[j] = e4[j] = 0;
                        if (mk) {
                            const int src = __ffsll((unsigned long long)mk) - 1;
                            mk &= mk - 1;
                            s4[j] = __builtin_amdgcn_readlane(r.start, src);
                            e4[j] = __builtin_amdgcn_readlane(r.end, src);
                            cnt++;
                        }
                    }
                    if (CNT)
                        for (int j = 0; j < cnt; j++) npairs += (unsigned long long)(e4[j] - s4[j]);
                    float mx[4], my[4], mz[4], mu[4], mv[4], mw[4];
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        mx[j] = my[j] = mz[j] = mu[j] = mv[j] = mw[j] = 0.0f;
                        if (j < cnt) {
                            const int64_t m = s4[j] + lane < e4[j] ? s4[j] + lane : qm;
                            mx[j] = mload<O32>(T.x, m); my[j] = mload<O32>(T.y, m);
                            mz[j] = mload<O32>(T.z, m); mu[j] = mload<O32>(T.vx, m);
                            mv[j] = mload<O32>(T.vy, m); mw[j] = mload<O32>(T.vz, m);
                        }
                    }
                    float d4[4];
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        d4[j] = __builtin_huge_valf();
                        if (j < cnt) {
                            const float d = P.nowrap
                                ? phase_d2<false>(q.x, q.y, q.z, q.u, q.v, q.w, mx[j], my[j],
                                                  mz[j], mu[j], mv[j], mw[j], P.a, P.c, A.pp.L,
                                                  A.pp.h)
                                : phase_d2<true>(q.x, q.y, q.z, q.u, q.v, q.w, mx[j], my[j],
                                                 mz[j], mu[j], mv[j], mw[j], P.a, P.c, A.pp.L,
                                                 A.pp.h);
                            if (s4[j] + lane < e4[j]) d4[j] = d;
                        }
                    }
                    bl = fminf(bl, fminf(fminf(d4[0], d4[1]), fminf(d4[2], d4[3])));
                    best = wmin_nonneg(bl);
                    if (best <= lo2) mk = 0;
                    // leaves still queued that the lowered `best` excludes
                    if (cull) mk &= __ballot(lb < best);
                }
                if (best <= lo2) {
                    sp = 0;
                    break;
                }
            }
        }
        if (lane == 0) {
            float out = best;
            if (brk) out = best <= lo2 ? 0.0f : (best <= P.hi2 ? best : __builtin_huge_valf());
            else if (mode == 3 && best <= lo3) out = 0.0f;
            else if (mode == 4 && !(best <= cap4)) out = __builtin_huge_valf();
            d2out[qm] = out;
        }
    }
    if (CNT && lane == 0 && npairs) atomicAdd(&g_nn_pairs[blockIdx.x & 63], npairs);
}

// ---------------------------------------------------------------------------
// host: build the tree of one level and run the traversals
// ---------------------------------------------------------------------------

__global__ void k_tree_roots(int nv, const LNode* __restrict__ nodes, TreeBuf tb,
                             int32_t* __restrict__ root) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    tb.istart[v] = (int32_t)nodes[v].t_off;
    tb.iend[v] = (int32_t)(nodes[v].t_off + nodes[v].size);
    tb.ientry[v] = -1;
    root[v] = v;
}

int tree_build(TreeBuf& tb, int32_t* root, const uint64_t* skeys, const LNode* nodes, int nv,
               const Members& T, const int32_t* mnode, const LParam* prm,
               const PhaseParams& pp, std::vector<int32_t>* level_begin, bool* overflow,
               int32_t* n_entry_out, hipStream_t st) {
    *overflow = false;
    *n_entry_out = 0;
    int32_t* hc = nullptr;
    RS_TRY(host_scratch((void**)&hc, 64));
    RS_HIP(hipMemsetAsync(tb.n_entry, 0, sizeof(int32_t), st));
    RS_HIP(hipMemsetAsync(tb.overflow, 0, sizeof(int32_t), st));
    RS_TRY(fill_i32(tb.n_inode, nv, 1, st));
    k_tree_roots<<<grid_for(nv, 64), 64, 0, st>>>(nv, nodes, tb, root);
    RS_HIP(hipGetLastError());
    level_begin->clear();
    int32_t b = 0, e = nv;
    for (int level = 0; level <= TREE_LEVELS; level++) {
        level_begin->push_back(b);
        if (e > b) {
            k_tree_split<<<(e - b + SPLIT_WAVES - 1) / SPLIT_WAVES, 64 * SPLIT_WAVES, 0, st>>>(
                skeys, b, e, level, tb);
            RS_HIP(hipGetLastError());
        }
        RS_HIP(hipMemcpyAsync(hc, tb.n_inode, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        RS_HIP(hipMemcpyAsync(hc + 1, tb.overflow, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        RS_HIP(hipStreamSynchronize(st));
        if (hc[1]) {
            *overflow = true;
            return RS_OK;
        }
        b = e;
        e = hc[0];
        if (e == b) break;
    }
    level_begin->push_back(b);
    RS_HIP(hipMemcpyAsync(hc, tb.n_entry, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    const int32_t n_entry = hc[0];
    if (n_entry > 0) {
        k_tree_leafbox<<<(n_entry + 3) / 4, 256, 0, st>>>(n_entry, tb, T, mnode, prm, pp);
        RS_HIP(hipGetLastError());
    }
    // internal boxes, deepest level first
    for (int l = (int)level_begin->size() - 2; l >= 0; l--) {
        int32_t lb = (*level_begin)[l], le = (*level_begin)[l + 1];
        if (le > lb) {
            k_tree_nodebox<<<(le - lb + 3) / 4, 256, 0, st>>>(lb, le, tb);
            RS_HIP(hipGetLastError());
        }
    }
    *n_entry_out = n_entry;
    return RS_OK;
}

int tree_refit_active(TreeBuf& tb, int32_t n_entry, const std::vector<int32_t>& level_begin,
                      const Members& T, const int32_t* mnode, const LParam* prm,
                      const PhaseParams& pp, const float* d2, hipStream_t st) {
    if (n_entry > 0) {
        k_tree_leafbox_active<<<(n_entry + 3) / 4, 256, 0, st>>>(n_entry, tb, T, mnode, prm, pp,
                                                                 d2);
        RS_HIP(hipGetLastError());
    }
    for (int l = (int)level_begin.size() - 2; l >= 0; l--) {
        int32_t lb = level_begin[l], le = level_begin[l + 1];
        if (le > lb) {
            k_tree_nodebox<<<(le - lb + 3) / 4, 256, 0, st>>>(lb, le, tb);
            RS_HIP(hipGetLastError());
        }
    }
    return RS_OK;
}

int tree_nn(const TArgs& A, int ntiles, float* d2, hipStream_t st) {
    const int c = xcd_chunk(ntiles);
    const bool o32 = use_o32(A.nmem);
    if (!prof_count_pairs()) {
        if (o32) k_tree_nn<true, false><<<xcd_chunk_grid(ntiles, c), 64, 0, st>>>(A, ntiles, c, d2);
        else k_tree_nn<false, false><<<xcd_chunk_grid(ntiles, c), 64, 0, st>>>(A, ntiles, c, d2);
        RS_HIP(hipGetLastError());
        return RS_OK;
    }
    // counting build: counters cleared before, read back after (synchronous)
    unsigned long long h[64] = {0};
    RS_HIP(hipStreamSynchronize(st));
    RS_HIP(hipMemcpyToSymbol(HIP_SYMBOL(g_nn_pairs), h, sizeof(h)));
    if (o32) k_tree_nn<true, true><<<xcd_chunk_grid(ntiles, c), 64, 0, st>>>(A, ntiles, c, d2);
    else k_tree_nn<false, true><<<xcd_chunk_grid(ntiles, c), 64, 0, st>>>(A, ntiles, c, d2);
    RS_HIP(hipGetLastError());
    RS_HIP(hipMemcpyFromSymbolAsync(h, HIP_SYMBOL(g_nn_pairs), sizeof(h), 0,
                                    hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    double sum = 0.0;
    for (int i = 0; i < 64; i++) sum += (double)h[i];
    prof_add_count("pairs_nn", sum);
    return RS_OK;
}

}  // namespace rs
