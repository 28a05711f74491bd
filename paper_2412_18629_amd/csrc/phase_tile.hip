// phase_tile.hip -- tile-cooperative searches over the 6D tree.
//
// One wavefront owns a tile of 64 consecutive members (one query per lane).
// It walks the tree ONCE with the bounding box of its queries, collecting
// every leaf that any query could need into an LDS list.  Each listed leaf
// is then loaded once (one member per lane) and only the queries whose own
// exact bound admits the leaf are replayed against it: each such query is
// broadcast to the lanes, every lane evaluates the pair with its member.
// Candidate data is read once per tile instead of once per query.  The walk
// scans up to four stack entries per pass (cells average about ten
// children), and linked pairs are united in batches of 64.
#include <type_traits>

#include "phase_common.h"

namespace rs {

// LDS per wavefront stays under 5 KB, so that eight wavefronts fit per SIMD:
// the link is bound by the latency of its walks and replays, and more
// resident wavefronts hide more of it than larger buffers save
constexpr int TSTACK = 520;   // >= 64 internal children x 8 levels
constexpr int TLIST = 96;     // candidate leaves buffered before processing (>= 64)
constexpr int THITS = 64;     // linked pairs buffered before their unions (>= 64)
static_assert(TLIST >= 64 && THITS >= 64, "one pass adds up to 64 leaves or pairs");

struct TileRec {
    float lo[6], hi[6];
    int32_t start, end, cfirst, ccount;
};

RS_DEV TileRec trec_load(const float* __restrict__ erec, int32_t k) {
    const float4* p = reinterpret_cast<const float4*>(erec + 16 * (int64_t)k);
    float4 a = p[0], b = p[1], c = p[2], d = p[3];
    TileRec r;
    r.lo[0] = a.x; r.lo[1] = a.y; r.lo[2] = a.z; r.lo[3] = a.w; r.lo[4] = b.x; r.lo[5] = b.y;
    r.hi[0] = b.z; r.hi[1] = b.w; r.hi[2] = c.x; r.hi[3] = c.y; r.hi[4] = c.z; r.hi[5] = c.w;
    r.start = __float_as_int(d.x);
    r.end = __float_as_int(d.y);
    r.cfirst = __float_as_int(d.z);
    r.ccount = __float_as_int(d.w);
    return r;
}

// exact lower bound of the computed d^2 between a point (w: unwrapped
// position, u: velocity) or a box (wlo..whi, ulo..uhi) and a record's box;
// the record's position box is stored widened by the slack that covers the
// rounding of the coordinates relative to the reference member, of the pair
// difference and of the image shift; velocity gaps and the bound lose a
// relative margin
RS_DEV float box_box_lb(const float blo[6], const float bhi[6], const TileRec& r, float a,
                        float c) {
    float sp = 0.0f, sv = 0.0f;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const float g = fmaxf(fmaxf(r.lo[d] - bhi[d], blo[d] - r.hi[d]), 0.0f);
        sp += g * g;
        float h = fmaxf(fmaxf(r.lo[3 + d] - bhi[3 + d], blo[3 + d] - r.hi[3 + d]), 0.0f) *
                  0.99999905f;
        sv += h * h;
    }
    return (a * sp + c * sv) * 0.99999f;
}

RS_DEV float tw_min(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

RS_DEV float tw_max(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

struct TStackEnt {
    int32_t cfirst, ccount;
};

// value of lane src (uniform) in every lane, through the scalar unit
RS_DEV float bcast(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Links within l among later members.  One wavefront per tile of 64
// consecutive members of one node (tiles never straddle nodes).  Pairs found
// within l are queued in LDS and united 64 at a time, one pair per lane, so
// that the union-find walks of many pairs are in flight together instead of
// one or two lanes walking while the rest of the wavefront waits.
// pair tests of the counting build (instrumentation level 2)
__device__ unsigned long long g_link_pairs[64];

template <bool O32, bool CNT>
__global__ void __launch_bounds__(64)
k_tile_link(TArgs A, int ntiles, int chunk, const float* __restrict__ d2,
            int32_t* __restrict__ par) {
    __shared__ TStackEnt stk[TSTACK];
    __shared__ int32_t list[TLIST];
    __shared__ int2 hits[THITS];
    const int lane = threadIdx.x;
    const int t = xcd_chunk_index(blockIdx.x, chunk);
    if (t >= ntiles) return;
    const TreeBuf& tb = A.tb;
    const int v = A.tile_node[t];
    const LNode nd = A.nodes[v];
    const int64_t ts = nd.t_off + 64ll * (t - nd.tile0);
    const int64_t te = min(ts + 64, nd.t_off + (int64_t)nd.size);
    const LParam P = A.prm[v];
    const Members& T = A.T;
    const PhaseParams& pp = A.pp;
    const float l2 = P.l2;
    const bool cull = P.cull != 0;

    // this lane's query
    const int64_t mq = ts + lane;
    const bool valid = mq < te;
    const int64_t mm = valid ? mq : ts;
    const float qx = mload<O32>(T.x, mm), qy = mload<O32>(T.y, mm), qz = mload<O32>(T.z, mm);
    const float qu = mload<O32>(T.vx, mm), qv = mload<O32>(T.vy, mm), qw = mload<O32>(T.vz, mm);
    const bool act = valid && mload<O32>(d2, mm) <= l2;
    const uint64_t amask = __ballot(act);
    if (!amask) return;
    const float w[3] = {min_image(qx - P.rx, pp.L, pp.h), min_image(qy - P.ry, pp.L, pp.h),
                        min_image(qz - P.rz, pp.L, pp.h)};
    const float qpt[6] = {w[0], w[1], w[2], qu, qv, qw};
    // box of the active queries
    float blo[6], bhi[6];
#pragma unroll
    for (int d = 0; d < 6; d++) {
        blo[d] = tw_min(act ? qpt[d] : __builtin_huge_valf());
        bhi[d] = tw_max(act ? qpt[d] : -__builtin_huge_valf());
    }
    const int64_t first_act = ts + __ffsll((unsigned long long)amask) - 1;

    int nhit = 0;
    unsigned long long npairs = 0;   // counting build only
    auto unite_hits = [&]() {
        __syncthreads();
        for (int i = lane; i < nhit; i += 64) uf_unite(par, hits[i].x, hits[i].y);
        nhit = 0;
        __syncthreads();
    };

    // one pass over the buffered candidate leaves: per leaf, the queries
    // whose own bound admits it are replayed against its members.  The pair
    // test runs on every lane (a lane past the leaf's end holds a valid
    // member and is masked afterwards), so the replay has no divergent branch.
    auto process = [&](int n, auto nowrap) {
        constexpr bool NOWRAP = decltype(nowrap)::value;
        for (int li = 0; li < n; li++) {
            const TileRec r = trec_load(tb.erec, list[li]);
            bool need = act && r.end > mq + 1;
            if (need && cull) need = !(box_box_lb(qpt, qpt, r, P.a, P.c) > l2);
            uint64_t mk = __ballot(need);
            if (!mk) continue;
            const int64_t mj = r.start + lane;
            const bool has = mj < r.end;
            const int64_t mjj = has ? mj : r.start;
            const float xj = mload<O32>(T.x, mjj), yj = mload<O32>(T.y, mjj),
                        zj = mload<O32>(T.z, mjj);
            const float uj = mload<O32>(T.vx, mjj), vj = mload<O32>(T.vy, mjj),
                        wj = mload<O32>(T.vz, mjj);
            // pairs are taken with later members only: for query ts + src the
            // lanes holding later members are those above src + ts - r.start
            const uint64_t hasm = __builtin_amdgcn_ballot_w64(has);
            const int32_t off = (int32_t)(ts + 1) - __builtin_amdgcn_readfirstlane(r.start);
            while (mk) {
                const int src = __ffsll((unsigned long long)mk) - 1;
                mk &= mk - 1;
                const float bx = bcast(qx, src), by = bcast(qy, src), bz = bcast(qz, src);
                const float bu = bcast(qu, src), bv = bcast(qv, src), bw = bcast(qw, src);
                const float dd = phase_d2<!NOWRAP>(bx, by, bz, bu, bv, bw, xj, yj, zj, uj, vj,
                                                   wj, P.a, P.c, pp.L, pp.h);
                const int32_t k0 = off + src;
                const uint64_t later = k0 <= 0 ? hasm : (k0 >= 64 ? 0ull : hasm & (~0ull << k0));
                if (CNT) npairs += (unsigned long long)__popcll(later);
                const uint64_t hm = later & __builtin_amdgcn_ballot_w64(dd <= l2);
                if (hm) {
                    if (nhit + __popcll(hm) > THITS) unite_hits();
                    if ((hm >> lane) & 1)
                        hits[nhit + __popcll(hm & lanemask_lt())] =
                            make_int2((int)(ts + src), (int)mj);
                    nhit += __popcll(hm);
                }
            }
        }
    };

    // walk the tree with the tile box; buffer leaves, flush when full
    int nlist = 0;
    if (lane == 0) stk[0] = TStackEnt{tb.cfirst[A.root[v]], tb.ccount[A.root[v]]};
    int sp = 1;
    __syncthreads();
    while (sp > 0) {
        // cells average about ten children: up to four entries whose
        // children fit in 64 lanes are scanned in one pass, each on its own
        // run of lanes (a pass pushes at most 64 entries, as one cell does)
        sp--;
        TStackEnt se = stk[sp];
        int32_t cf1 = 0, cf2 = 0, cf3 = 0, e1 = 64, e2 = 64, e3 = 64, tot = se.ccount;
        if (tot <= 64) {
            if (sp > 0 && tot + stk[sp - 1].ccount <= 64) {
                cf1 = stk[--sp].cfirst;
                e1 = tot;
                tot += stk[sp].ccount;
                if (sp > 0 && tot + stk[sp - 1].ccount <= 64) {
                    cf2 = stk[--sp].cfirst;
                    e2 = tot;
                    tot += stk[sp].ccount;
                    if (sp > 0 && tot + stk[sp - 1].ccount <= 64) {
                        cf3 = stk[--sp].cfirst;
                        e3 = tot;
                        tot += stk[sp].ccount;
                    }
                }
            }
            // lanes [0, e1) scan the first entry, [e1, e2) the second, ...
            se.ccount = tot;
        }
        __syncthreads();
        for (int32_t b0 = 0; b0 < se.ccount; b0 += 64) {
            const int32_t k = lane >= e3   ? cf3 + lane - e3
                              : lane >= e2 ? cf2 + lane - e2
                              : lane >= e1 ? cf1 + lane - e1
                                           : se.cfirst + b0 + lane;
            bool need = false, leaf = false;
            TileRec r;
            r.cfirst = -1;
            r.ccount = 0;
            if (b0 + lane < se.ccount) {
                r = trec_load(tb.erec, k);
                leaf = r.cfirst < 0;
                need = r.end > first_act + 1 &&
                       (!cull || !(box_box_lb(blo, bhi, r, P.a, P.c) > l2));
            }
            const uint64_t imask = __ballot(need && !leaf);
            if (need && !leaf)
                stk[sp + __popcll(imask & lanemask_lt())] = TStackEnt{r.cfirst, r.ccount};
            sp += __popcll(imask);
            const uint64_t lmask = __ballot(need && leaf);
            if (nlist + __popcll(lmask) > TLIST) {
                __syncthreads();
                if (P.nowrap) process(nlist, std::true_type{});
                else process(nlist, std::false_type{});
                nlist = 0;
            }
            if (need && leaf) list[nlist + __popcll(lmask & lanemask_lt())] = k;
            nlist += __popcll(lmask);
            __syncthreads();
        }
    }
    if (P.nowrap) process(nlist, std::true_type{});
    else process(nlist, std::false_type{});
    unite_hits();
    if (CNT && lane == 0 && npairs) atomicAdd(&g_link_pairs[blockIdx.x & 63], npairs);
}

int tile_link(const TArgs& A, int ntiles, const float* d2, int32_t* par, hipStream_t st) {
    if (ntiles <= 0) return RS_OK;
    const int c = xcd_chunk(ntiles);
    const bool o32 = use_o32(A.nmem);
    const unsigned grid = xcd_chunk_grid(ntiles, c);
    if (!prof_count_pairs()) {
        if (o32) k_tile_link<true, false><<<grid, 64, 0, st>>>(A, ntiles, c, d2, par);
        else k_tile_link<false, false><<<grid, 64, 0, st>>>(A, ntiles, c, d2, par);
        RS_HIP(hipGetLastError());
        return RS_OK;
    }
    // counting build: counters cleared before, read back after (synchronous)
    unsigned long long h[64] = {0};
    RS_HIP(hipStreamSynchronize(st));
    RS_HIP(hipMemcpyToSymbol(HIP_SYMBOL(g_link_pairs), h, sizeof(h)));
    if (o32) k_tile_link<true, true><<<grid, 64, 0, st>>>(A, ntiles, c, d2, par);
    else k_tile_link<false, true><<<grid, 64, 0, st>>>(A, ntiles, c, d2, par);
    RS_HIP(hipGetLastError());
    RS_HIP(hipMemcpyFromSymbolAsync(h, HIP_SYMBOL(g_link_pairs), sizeof(h), 0,
                                    hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    double sum = 0.0;
    for (int i = 0; i < 64; i++) sum += (double)h[i];
    prof_add_count("pairs_link", sum);
    return RS_OK;
}

}  // namespace rs
