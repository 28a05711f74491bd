// phase_large.hip -- one recursion level of the 6D split for nodes too large
// for a single workgroup's LDS (more than SMALL_MAX members).
//
// All large nodes of a level are processed together:
//   moments   per (node, chunk) work items -> global 128-bit accumulators
//   keys      6D Morton code of the normalised, centred coordinates (a
//             monotone log-like squash per axis); node rank in the top bits
//   sort      key/index radix sort -> members of a node are contiguous and
//             6D-local; 64 consecutive members form a tile, 64 tiles a
//             super-tile, whose boxes decide whether a node may be culled
//   tree      6D Morton-prefix search tree with exact boxes (phase_tree.hip)
//   NN        per query, a depth-first search of its node's tree, bounded
//             by the exact box lower bound (bracketed when a proposal is
//             given, then verified and refined)
//   select    per-node 4-pass radix select of the k-th smallest d^2
//   link      one wavefront per tile: one tree walk with the tile's box,
//             replays of the admitted leaves (phase_tile.hip); global
//             lock-free union-find
//   children  components of >= min_sub members (not the whole node): small
//             ones go to the workgroup-subtree kernel, large ones to the
//             next level
// Bounding-box culling only removes pairs whose computed d^2 provably cannot
// matter (slack covers every fp32 rounding of the coordinates and the
// metric); nodes spanning more than a quarter box per axis are not culled.
#include "phase_common.h"

#include <stdlib.h>

namespace rs {




// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256)
k_lmom(const LItem* __restrict__ items, const LNode* __restrict__ nodes, Members in,
       const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z,
       PhaseParams pp, unsigned long long* __restrict__ gacc, uint32_t* __restrict__ gext) {
    __shared__ unsigned long long acc[18];
    __shared__ uint32_t ext[6];
    const LItem it = items[blockIdx.x];
    const LNode nd = nodes[it.v];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < 18) acc[tid] = 0;
    if (tid < 3) ext[tid] = 0xffffffffu;
    else if (tid < 6) ext[tid] = 0;
    __syncthreads();
    int64_t qref[3] = {quant_pos(X[nd.minidx]), quant_pos(Y[nd.minidx]), quant_pos(Z[nd.minidx])};
    Moments mo;
    mom_zero(mo);
    uint32_t mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, mx[3] = {0, 0, 0};
    for (int j = tid; j < it.len; j += 256) {
        int64_t g = it.in_start + j;
        float p[3] = {in.x[g], in.y[g], in.z[g]};
        mom_add(mo, p[0], p[1], p[2], in.vx[g], in.vy[g], in.vz[g], qref, pp.LQ);
#pragma unroll
        for (int ax = 0; ax < 3; ax++) {
            uint32_t b = __float_as_uint(p[ax]);
            mn[ax] = b < mn[ax] ? b : mn[ax];
            mx[ax] = b > mx[ax] ? b : mx[ax];
        }
    }
    if (wave * 64 < it.len) {
        mom_wave_reduce(mo);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
            for (int ax = 0; ax < 3; ax++) {
                uint32_t o1 = (uint32_t)__shfl_xor((int)mn[ax], off, 64);
                uint32_t o2 = (uint32_t)__shfl_xor((int)mx[ax], off, 64);
                mn[ax] = o1 < mn[ax] ? o1 : mn[ax];
                mx[ax] = o2 > mx[ax] ? o2 : mx[ax];
            }
        if (lane == 0) {
            mom_accumulate(acc, mo);
            for (int ax = 0; ax < 3; ax++) {
                atomicMin(ext + ax, mn[ax]);
                atomicMax(ext + 3 + ax, mx[ax]);
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long* g = gacc + 18 * (int64_t)it.v;
        for (int q = 0; q < 6; q++) atomicAdd(g + q, acc[q]);
        for (int q = 0; q < 6; q++) {
            u128 v = ((u128)acc[7 + 2 * q] << 64) | (u128)acc[6 + 2 * q];
            acc_add128(g + 6 + 2 * q, g + 7 + 2 * q, v);
        }
        for (int ax = 0; ax < 3; ax++) {
            atomicMin(gext + 6 * it.v + ax, ext[ax]);
            atomicMax(gext + 6 * it.v + 3 + ax, ext[3 + ax]);
        }
    }
}

__global__ void k_lnorm(int nv, const LNode* __restrict__ nodes,
                        const unsigned long long* __restrict__ gacc,
                        const uint32_t* __restrict__ gext, const float* __restrict__ X,
                        const float* __restrict__ Y, const float* __restrict__ Z,
                        PhaseParams pp, NodeRec nr, LParam* __restrict__ prm) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const LNode nd = nodes[v];
    Norm nm = mom_finalize(gacc + 18 * (int64_t)v, nd.size);
    LParam P;
    P.a = nm.a;
    P.c = nm.c;
    P.sa = sqrtf(nm.a);
    P.sc = sqrtf(nm.c);
    P.rx = X[nd.minidx];
    P.ry = Y[nd.minidx];
    P.rz = Z[nd.minidx];
    P.cx = (float)((double)P.rx + nm.mean[0]);
    P.cy = (float)((double)P.ry + nm.mean[1]);
    P.cz = (float)((double)P.rz + nm.mean[2]);
    P.cu = (float)nm.mean[3];
    P.cv = (float)nm.mean[4];
    P.cw = (float)nm.mean[5];
    bool nowrap = true;
    for (int ax = 0; ax < 3; ax++) {
        float e = __uint_as_float(gext[6 * v + 3 + ax]) - __uint_as_float(gext[6 * v + ax]);
        nowrap = nowrap && (e <= pp.h);
    }
    P.nowrap = nowrap ? 1 : 0;
    P.cull = 0;
    P.pf = 0;
    P.pm = 0;
    P.kk = (int32_t)select_rank(nd.size, pp.f_ppm);
    P.l2 = 0.0f;
    P.nnmode = 0;
    P.lo2 = 0.0f;
    P.hi2 = 0.0f;
    P.isx = nm.sx2 > 0.0f ? 1.0f / sqrtf(nm.sx2) : 0.0f;
    P.isv = nm.sv2 > 0.0f ? 1.0f / sqrtf(nm.sv2) : 0.0f;
    prm[v] = P;
    nr.a[nd.slot] = nm.a;
    nr.c[nd.slot] = nm.c;
    nr.sx2[nd.slot] = nm.sx2;
    nr.sv2[nd.slot] = nm.sv2;
}

// squash a normalised coordinate into [0, 128): finer near the centre,
// sign(u) log2(1 + 8|u|) / 5 clamped to [-1, 1].  The key only orders the
// members for the search tree (any monotone squash gives the same results),
// so the hardware base-2 logarithm serves.
RS_DEV uint32_t squash7(float u) {
    float t = copysignf(__log2f(1.0f + 8.0f * fabsf(u)) * 0.2f, u);
    t = fminf(fmaxf(t, -1.0f), 1.0f);
    int q = (int)((t + 1.0f) * 63.999f);
    return (uint32_t)(q < 0 ? 0 : (q > 127 ? 127 : q));
}

// the 7 bits of v moved to bit positions 0, 6, 12, ..., 36 (bit k by 5k,
// in three shift-and-mask steps: by 20 for k >= 4, by 10 for k in {2, 3, 6},
// by 5 for odd k)
RS_DEV uint64_t spread7(uint32_t v) {
    uint64_t x = v & 0x7fu;
    x = (x | (x << 20)) & 0x000000000700000Full;
    x = (x | (x << 10)) & 0x0000001003003003ull;
    x = (x | (x << 5)) & 0x0000001041041041ull;
    return x;
}

// 42-bit Morton code of six 7-bit coordinates: bit b of coordinate d at
// position 6b + 5 - d
RS_DEV uint64_t morton6(const uint32_t q[6]) {
    uint64_t k = 0;
#pragma unroll
    for (int d = 0; d < 6; d++) k |= spread7(q[d]) << (5 - d);
    return k;
}

// Morton keys of the level's members (node rank above them), and each
// member's coordinates and index interleaved at its position t, 28 bytes a
// member, so that the gather in Morton order fetches one record (one or two
// cache lines) per member instead of seven scattered values
__global__ void __launch_bounds__(256)
k_lkeys(const LItem* __restrict__ items, Members in, const LParam* __restrict__ prm,
        PhaseParams pp, uint64_t* __restrict__ keys, int32_t* __restrict__ src,
        float* __restrict__ rec) {
    const LItem it = items[blockIdx.x];
    const LParam P = prm[it.v];
    for (int j = threadIdx.x; j < it.len; j += 256) {
        int64_t g = it.in_start + j;
        const float x = in.x[g], y = in.y[g], z = in.z[g];
        const float vx = in.vx[g], vy = in.vy[g], vz = in.vz[g];
        uint32_t q[6];
        q[0] = squash7(min_image(x - P.cx, pp.L, pp.h) * P.sa);
        q[1] = squash7(min_image(y - P.cy, pp.L, pp.h) * P.sa);
        q[2] = squash7(min_image(z - P.cz, pp.L, pp.h) * P.sa);
        q[3] = squash7((vx - P.cu) * P.sc);
        q[4] = squash7((vy - P.cv) * P.sc);
        q[5] = squash7((vz - P.cw) * P.sc);
        int64_t t = it.t_start + j;
        keys[t] = ((uint64_t)it.v << 42) | morton6(q);
        src[t] = (int32_t)t;
        float* r = rec + 7 * t;
        r[0] = x;
        r[1] = y;
        r[2] = z;
        r[3] = vx;
        r[4] = vy;
        r[5] = vz;
        r[6] = __int_as_float(in.idx[g]);
    }
}

__global__ void k_lgather(int64_t m, const int32_t* __restrict__ perm,
                          const uint64_t* __restrict__ skeys, const float* __restrict__ rec,
                          Members out, int32_t* __restrict__ mnode) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= m) return;
    const float* r = rec + 7 * (int64_t)perm[t];
    out.x[t] = r[0];
    out.y[t] = r[1];
    out.z[t] = r[2];
    out.vx[t] = r[3];
    out.vy[t] = r[4];
    out.vz[t] = r[5];
    out.idx[t] = __float_as_int(r[6]);
    mnode[t] = (int32_t)(skeys[t] >> 42);
}

RS_DEV void tile_range(const LNode& nd, int t, int64_t* ts, int64_t* te) {
    int64_t s = nd.t_off + 64ll * (t - nd.tile0);
    int64_t e = s + 64;
    int64_t end = nd.t_off + nd.size;
    *ts = s;
    *te = e < end ? e : end;
}

RS_DEV float wave_min(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

RS_DEV float wave_max(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// tile boxes: [lo wx wy wz u v w, hi wx wy wz u v w]
__global__ void __launch_bounds__(64)
k_ltbox(const int32_t* __restrict__ tile_node, const LNode* __restrict__ nodes, Members T,
        const LParam* __restrict__ prm, PhaseParams pp, float* __restrict__ tbox) {
    const int t = blockIdx.x, lane = threadIdx.x;
    const int v = tile_node[t];
    const LNode nd = nodes[v];
    const LParam P = prm[v];
    int64_t ts, te;
    tile_range(nd, t, &ts, &te);
    int64_t m = ts + lane;
    bool ok = m < te;
    float c[6];
    if (ok) {
        c[0] = min_image(T.x[m] - P.rx, pp.L, pp.h);
        c[1] = min_image(T.y[m] - P.ry, pp.L, pp.h);
        c[2] = min_image(T.z[m] - P.rz, pp.L, pp.h);
        c[3] = T.vx[m];
        c[4] = T.vy[m];
        c[5] = T.vz[m];
    }
#pragma unroll
    for (int d = 0; d < 6; d++) {
        float lo = wave_min(ok ? c[d] : __builtin_huge_valf());
        float hi = wave_max(ok ? c[d] : -__builtin_huge_valf());
        if (lane == 0) {
            tbox[12 * (int64_t)t + d] = lo;
            tbox[12 * (int64_t)t + 6 + d] = hi;
        }
    }
}

__global__ void __launch_bounds__(64)
k_lsbox(const int32_t* __restrict__ super_node, const LNode* __restrict__ nodes,
        const float* __restrict__ tbox, float* __restrict__ sbox) {
    const int s = blockIdx.x, lane = threadIdx.x;
    const LNode nd = nodes[super_node[s]];
    int t0 = nd.tile0 + 64 * (s - nd.super0);
    int t1 = t0 + 64;
    if (t1 > nd.tile0 + nd.ntile) t1 = nd.tile0 + nd.ntile;
    int t = t0 + lane;
    bool ok = t < t1;
#pragma unroll
    for (int d = 0; d < 6; d++) {
        float lo = wave_min(ok ? tbox[12 * (int64_t)t + d] : __builtin_huge_valf());
        float hi = wave_max(ok ? tbox[12 * (int64_t)t + 6 + d] : -__builtin_huge_valf());
        if (lane == 0) {
            sbox[12 * (int64_t)s + d] = lo;
            sbox[12 * (int64_t)s + 6 + d] = hi;
        }
    }
}

// culling is allowed when every pair's min-image difference is the
// difference of the unwrapped coordinates: extent below a quarter box
__global__ void k_lcull(int nv, const LNode* __restrict__ nodes, const float* __restrict__ sbox,
                        PhaseParams pp, LParam* __restrict__ prm) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const LNode nd = nodes[v];
    float lo[3] = {1e30f, 1e30f, 1e30f}, hi[3] = {-1e30f, -1e30f, -1e30f};
    for (int s = nd.super0; s < nd.super0 + nd.nsuper; s++)
        for (int d = 0; d < 3; d++) {
            lo[d] = fminf(lo[d], sbox[12 * (int64_t)s + d]);
            hi[d] = fmaxf(hi[d], sbox[12 * (int64_t)s + 6 + d]);
        }
    bool ok = true;
    for (int d = 0; d < 3; d++) ok = ok && (hi[d] - lo[d] <= 0.5f * pp.h);
    prm[v].cull = ok ? 1 : 0;
}

// ---------------------------------------------------------------------------
// per-node radix select over the d^2 bit patterns
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256)
k_lhist(const LItem* __restrict__ items, const float* __restrict__ d2,
        const LParam* __restrict__ prm, int shift, int32_t* __restrict__ ghist) {
    __shared__ int32_t hist[256];
    const LItem it = items[blockIdx.x];
    const LParam P = prm[it.v];
    hist[threadIdx.x] = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < it.len; j += 256) {
        uint32_t u = __float_as_uint(d2[it.t_start + j]);
        if ((u & P.pm) == P.pf) atomicAdd(hist + ((u >> shift) & 255u), 1);
    }
    __syncthreads();
    int h = hist[threadIdx.x];
    if (h) atomicAdd(ghist + 256 * (int64_t)it.v + threadIdx.x, h);
}

__global__ void __launch_bounds__(64)
k_lpick(const int32_t* __restrict__ ghist, int shift, LParam* __restrict__ prm,
        const LNode* __restrict__ nodes, NodeRec nr, int last) {
    const int v = blockIdx.x, lane = threadIdx.x;
    const int32_t* hh = ghist + 256 * (int64_t)v;
    int h0 = hh[4 * lane], h1 = hh[4 * lane + 1], h2 = hh[4 * lane + 2], h3 = hh[4 * lane + 3];
    int tot = h0 + h1 + h2 + h3, inc = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    int before = inc - tot;
    int kk = prm[v].kk;
    if (before < kk && kk <= inc) {
        int k2 = kk - before, b = 4 * lane;
        if (k2 > h0) { k2 -= h0; b++;
            if (k2 > h1) { k2 -= h1; b++;
                if (k2 > h2) { k2 -= h2; b++; } } }
        uint32_t pf = prm[v].pf | ((uint32_t)b << shift);
        prm[v].pf = pf;
        prm[v].pm |= 255u << shift;
        prm[v].kk = k2;
        if (last) {
            prm[v].l2 = __uint_as_float(pf);
            nr.l2[nodes[v].slot] = __uint_as_float(pf);
        }
    }
}

// ---------------------------------------------------------------------------
// linking within l
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// components and children
// ---------------------------------------------------------------------------

__global__ void k_liota(int64_t m, int32_t* __restrict__ par) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < m) par[t] = (int32_t)t;
}

__global__ void k_lflat(int64_t m, int32_t* __restrict__ par, int32_t* __restrict__ cnt,
                        unsigned long long* __restrict__ mpk) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= m) return;
    par[t] = uf_root(par, (int)t);
    cnt[t] = 0;
    mpk[t] = ~0ull;
}

// component sizes and packed (index, slot) minima, aggregated per wavefront
// over runs of members sharing a root
__global__ void k_lstat(int64_t m, const int32_t* __restrict__ par,
                        const int32_t* __restrict__ idx, int32_t* __restrict__ cnt,
                        unsigned long long* __restrict__ mpk) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool active = t < m;
    const int32_t r = active ? par[t] : -1;
    const unsigned long long key =
        active ? (((unsigned long long)(uint32_t)idx[t] << 32) | (uint32_t)t) : ~0ull;
    uint64_t todo = __ballot(active);
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int32_t lr = __shfl(r, leader, 64);
        const bool mine = active && r == lr;
        const uint64_t grp = __ballot(mine);
        // a root held by one lane only (members that linked nothing in this
        // wavefront, about a third of them) needs no reduction
        const unsigned long long mn =
            __popcll(grp) == 1 ? key : wave_min_u64(mine ? key : ~0ull);
        if ((int)(threadIdx.x & 63) == leader) {
            atomicAdd(cnt + lr, __popcll(grp));
            atomicMin(mpk + lr, mn);
        }
        todo &= ~grp;
    }
}


__global__ void k_lchild(int64_t m, const int32_t* __restrict__ par,
                         const int32_t* __restrict__ cnt,
                         const unsigned long long* __restrict__ mpk,
                         const int32_t* __restrict__ mnode, const LNode* __restrict__ nodes,
                         PhaseParams pp, NodeRec nr, int32_t* __restrict__ cslot,
                         int64_t* __restrict__ coff, int32_t* __restrict__ cfill,
                         int8_t* __restrict__ cclass, LCounters* __restrict__ ctr,
                         SmallItem* __restrict__ small_items, ChildOut* __restrict__ large_out,
                         int64_t cap_m) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= m) return;
    if (par[t] != (int32_t)t) return;
    const LNode nd = nodes[mnode[t]];
    int c = cnt[t];
    cslot[t] = -1;
    if (c < pp.min_sub || c >= nd.size) return;
    int slot = atomicAdd(nr.count, 1);
    if (slot >= nr.cap) {
        atomicOr(nr.overflow, 1);
        return;
    }
    int minidx = (int)(mpk[t] >> 32);
    nr.level[slot] = nd.level + 1;
    nr.minidx[slot] = minidx;
    nr.parent[slot] = nd.slot;
    nr.size[slot] = c;
    int64_t off;
    if (c <= SMALL_MAX) {
        off = (int64_t)atomicAdd(&ctr->tot_small, (unsigned long long)c);
        int i = atomicAdd(&ctr->n_small, 1);
        small_items[i] = SmallItem{slot, nd.level + 1, c, minidx, off};
        cclass[t] = 0;
    } else {
        // large children fill the shared child buffer from its end
        off = cap_m - (int64_t)atomicAdd(&ctr->tot_large, (unsigned long long)c) - c;
        int i = atomicAdd(&ctr->n_large, 1);
        large_out[i] = ChildOut{slot, c, minidx, nd.level + 1, off};
        cclass[t] = 1;
    }
    coff[t] = off;
    cfill[t] = 0;
    cslot[t] = slot;
}

__global__ void k_lscatter(int64_t m, const int32_t* __restrict__ par, Members T,
                           const int32_t* __restrict__ cslot, const int64_t* __restrict__ coff,
                           int32_t* __restrict__ cfill, const int8_t* __restrict__ cclass,
                           Members S, Members N, int32_t* __restrict__ deepest) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int32_t r = t < m ? par[t] : -1;
    const int32_t s = r >= 0 ? cslot[r] : -1;
    const bool active = s >= 0;
    // slots within the child: one atomic per run of lanes with the same root
    int64_t pos = 0;
    uint64_t todo = __ballot(active);
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int32_t lr = __shfl(r, leader, 64);
        const bool mine = active && r == lr;
        const uint64_t grp = __ballot(mine);
        int base = 0;
        if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(cfill + lr, __popcll(grp));
        base = __shfl(base, leader, 64);
        if (mine) pos = coff[r] + base + __popcll(grp & lanemask_lt());
        todo &= ~grp;
    }
    if (!active) return;
    Members D = cclass[r] ? N : S;
    D.x[pos] = T.x[t];
    D.y[pos] = T.y[t];
    D.z[pos] = T.z[t];
    D.vx[pos] = T.vx[t];
    D.vy[pos] = T.vy[t];
    D.vz[pos] = T.vz[t];
    D.idx[pos] = T.idx[t];
    deepest[T.idx[t]] = s;
}

// ---------------------------------------------------------------------------
// proposer features, proposal and exact acceptance of the bracket
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256)
k_lfeat(const LItem* __restrict__ items, Members in, const LParam* __restrict__ prm,
        PhaseParams pp, int32_t* __restrict__ lhist) {
    __shared__ int32_t hist[16];
    const LItem it = items[blockIdx.x];
    const LParam P = prm[it.v];
    if (threadIdx.x < 16) hist[threadIdx.x] = 0;
    __syncthreads();
    FeatFrame f;
    f.cx = P.cx; f.cy = P.cy; f.cz = P.cz; f.cu = P.cu; f.cv = P.cv; f.cw = P.cw;
    f.isx = P.isx; f.isv = P.isv;
    for (int j = threadIdx.x; j < it.len; j += 256) {
        int64_t g = it.in_start + j;
        int br, bv;
        feat_member_bins(f, in.x[g], in.y[g], in.z[g], in.vx[g], in.vy[g], in.vz[g], pp.L, pp.h,
                         &br, &bv);
        atomicAdd(hist + br, 1);
        atomicAdd(hist + bv, 1);
    }
    __syncthreads();
    if (threadIdx.x < 16 && hist[threadIdx.x])
        atomicAdd(lhist + 16 * it.v + threadIdx.x, hist[threadIdx.x]);
}

__global__ void k_lfeat_fin(int nv, const LNode* __restrict__ nodes,
                            const unsigned long long* __restrict__ gacc,
                            const int32_t* __restrict__ lhist, float* __restrict__ lfeat,
                            NodeRec nr, int want_feat) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const LNode nd = nodes[v];
    float* f = lfeat + (int64_t)v * RS_NFEAT;
    feat_write(f, gacc + 18 * (int64_t)v, nd.size, nd.level, lhist + 16 * v);
    if (want_feat)
        for (int i = 0; i < RS_NFEAT; i++) nr.feat[(int64_t)nd.slot * RS_NFEAT + i] = f[i];
}

// bracket [0.95 l^, 1.05 l^] around the proposal, compared as squares
__global__ void k_lbracket(int nv, const float* __restrict__ lnl, LParam* __restrict__ prm) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    float l = expf(lnl[v]);
    if (!(l > 0.0f) || !(l < 3.0e18f)) {
        prm[v].nnmode = 0;
        return;
    }
    float lo = 0.95f * l, hi = 1.05f * l;
    prm[v].lo2 = lo * lo;
    prm[v].hi2 = hi * hi;
    prm[v].nnmode = 1;
}

// #(d <= lo) and #(d <= hi) of bracket-mode nodes (d encoded by the search:
// 0 = a neighbour within lo, exact in (lo, hi], +inf beyond hi)
__global__ void __launch_bounds__(256)
k_lcount(const LItem* __restrict__ items, const float* __restrict__ d2,
         const LParam* __restrict__ prm, int32_t* __restrict__ lcnt) {
    __shared__ int32_t c[2];
    const LItem it = items[blockIdx.x];
    if (prm[it.v].nnmode != 1) return;
    if (threadIdx.x < 2) c[threadIdx.x] = 0;
    __syncthreads();
    int a = 0, b = 0;
    for (int j = threadIdx.x; j < it.len; j += 256) {
        float d = d2[it.t_start + j];
        a += d == 0.0f;
        b += d < __builtin_huge_valf();
    }
    // wavefront sums first: one LDS atomic per wavefront, not per thread
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(c, a);
        atomicAdd(c + 1, b);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(lcnt + 2 * it.v, c[0]);
        atomicAdd(lcnt + 2 * it.v + 1, c[1]);
    }
}

// accept when #(<= lo) < k <= #(<= hi) (nnmode 2: done); otherwise the
// queries that can hold the k-th value are searched again exactly: those
// within lo when k <= #(<= lo) (nnmode 3), those beyond hi when
// k > #(<= hi) (nnmode 4)
__global__ void k_laccept(int nv, const int32_t* __restrict__ lcnt, LParam* __restrict__ prm,
                          int32_t* __restrict__ lstat) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv || prm[v].nnmode != 1) return;
    int k = prm[v].kk;
    bool ok = lcnt[2 * v] < k && k <= lcnt[2 * v + 1];
    prm[v].nnmode = ok ? 2 : (k <= lcnt[2 * v] ? 3 : 4);
    atomicAdd(lstat + (ok ? 0 : 1), 1);
}

// after the first refinement step: #(d = 0) of the nodes refined below lo,
// #(d < +inf) of those refined above hi
__global__ void __launch_bounds__(256)
k_lcount_refine(const LItem* __restrict__ items, const float* __restrict__ d2,
                const LParam* __restrict__ prm, int32_t* __restrict__ lcnt) {
    __shared__ int32_t c;
    const LItem it = items[blockIdx.x];
    const int mode = prm[it.v].nnmode;
    if (mode != 3 && mode != 4) return;
    if (threadIdx.x == 0) c = 0;
    __syncthreads();
    int b = 0;
    for (int j = threadIdx.x; j < it.len; j += 256) {
        const float d = d2[it.t_start + j];
        b += mode == 3 ? d == 0.0f : d < __builtin_huge_valf();
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) b += __shfl_xor(b, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(&c, b);
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(lcnt + 2 * it.v + (mode == 3 ? 0 : 1), c);
}

// the refinement is complete when the k-th value lies in the band the first
// step resolved exactly: #(d <= lo3) < k below lo, k <= #(d <= cap4) above
// hi; otherwise the second step (modes 6, 5) searches the rest
__global__ void k_laccept_refine(int nv, const int32_t* __restrict__ lcnt,
                                 LParam* __restrict__ prm, int32_t* __restrict__ lstat) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int mode = prm[v].nnmode;
    if (mode != 3 && mode != 4) return;
    const int k = prm[v].kk;
    const bool ok = mode == 3 ? lcnt[2 * v] < k : k <= lcnt[2 * v + 1];
    prm[v].nnmode = ok ? 2 : (mode == 3 ? 6 : 5);
    if (!ok) atomicAdd(lstat + 2, 1);
}

__global__ void k_lext_init(int nv, uint32_t* __restrict__ gext) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 6 * nv) gext[i] = (i % 6) < 3 ? 0xffffffffu : 0u;
}

__global__ void k_bucket(const SmallItem* __restrict__ in, int n, SmallItem* __restrict__ out,
                         int64_t stride, int32_t* __restrict__ bcount) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    SmallItem it = in[i];
    int b = it.size <= 64 ? 0 : it.size <= 256 ? 1 : it.size <= 1024 ? 2 : 3;   // small_bucket_of
    int p = atomicAdd(bcount + b, 1);
    out[b * stride + p] = it;
}

// ---------------------------------------------------------------------------
// host side of one level
// ---------------------------------------------------------------------------

// Bytes of the large-node work space for up to m members per pass.  Small
// children hold at least min_sub members each and are disjoint, so at most
// m / min_sub of them exist per level.
size_t large_work_bytes(int64_t m, int32_t min_sub) {
    int64_t nodes = m / (SMALL_MAX + 1) + 2;
    int64_t items = m / 4096 + nodes + 2;
    int64_t tiles = m / 64 + nodes + 2;
    int64_t supers = tiles / 64 + nodes + 2;
    int64_t small = m / (min_sub > 1 ? min_sub : 1) + 2;
    size_t b = 0;
    auto add = [&](size_t x) { b += arena_round(x); };
    for (int k = 0; k < 2 * 7; k++) add(4 * m);                 // T, SN
    add(8 * m); add(8 * m);                                     // keys
    add(4 * m); add(4 * m); add(4 * m);                         // src, perm, mnode
    add(28 * m);                                                // par..cfill, mpk, d2 (records)
    add(8 * m); add(m);                                         // coff, cclass
    add(sizeof(LNode) * nodes); add(sizeof(LItem) * items); add(sizeof(LParam) * nodes);
    add(8 * 18 * nodes); add(4 * 6 * nodes); add(4 * 256 * nodes);
    add(4 * tiles); add(4 * supers); add(4 * 12 * tiles); add(4 * 12 * supers);
    add(sizeof(LCounters)); add(sizeof(SmallItem) * small); add(sizeof(SmallItem) * 4 * small);
    add(64); add(sizeof(ChildOut) * nodes);
    add(sort_temp_bytes(m));
    add(4 * nodes); add(4 * 16 * nodes); add(4 * RS_NFEAT * nodes); add(4 * nodes);
    add(4 * 2 * nodes); add(64);
    return b + 4096;
}

int large_work_carve(Arena* ar, int64_t m, int32_t min_sub, LargeWork* w) {
    w->cap_m = m;
    w->cap_nodes = m / (SMALL_MAX + 1) + 2;
    w->cap_items = m / 4096 + w->cap_nodes + 2;
    w->cap_tiles = m / 64 + w->cap_nodes + 2;
    w->cap_supers = w->cap_tiles / 64 + w->cap_nodes + 2;
    w->cap_small = m / (min_sub > 1 ? min_sub : 1) + 2;
    Members* bufs[2] = {&w->T, &w->SN};
    for (Members* b : bufs) {
        b->x = take<float>(ar, m); b->y = take<float>(ar, m); b->z = take<float>(ar, m);
        b->vx = take<float>(ar, m); b->vy = take<float>(ar, m); b->vz = take<float>(ar, m);
        b->idx = take<int32_t>(ar, m);
    }
    w->kin = take<uint64_t>(ar, m);
    w->kout = take<uint64_t>(ar, m);
    w->src = take<int32_t>(ar, m);
    w->perm = take<int32_t>(ar, m);
    w->mnode = take<int32_t>(ar, m);
    // union-find, component and child tables and the NN distances share one
    // region: none is live from one level's end to its next level's gather,
    // which keeps the interleaved member records there (28 bytes a member)
    char* reg = take<char>(ar, 28 * (size_t)m);
    w->par = reinterpret_cast<int32_t*>(reg);
    w->cnt = reinterpret_cast<int32_t*>(reg + 4 * (size_t)m);
    w->cslot = reinterpret_cast<int32_t*>(reg + 8 * (size_t)m);
    w->cfill = reinterpret_cast<int32_t*>(reg + 12 * (size_t)m);
    w->mpk = reinterpret_cast<unsigned long long*>(reg + 16 * (size_t)m);
    w->d2 = reinterpret_cast<float*>(reg + 24 * (size_t)m);
    w->lrec = reinterpret_cast<float*>(reg);
    w->coff = take<int64_t>(ar, m);
    w->cclass = take<int8_t>(ar, m);
    w->nodes = take<LNode>(ar, w->cap_nodes);
    w->items = take<LItem>(ar, w->cap_items);
    w->prm = take<LParam>(ar, w->cap_nodes);
    w->gacc = take<unsigned long long>(ar, 18 * w->cap_nodes);
    w->gext = take<uint32_t>(ar, 6 * w->cap_nodes);
    w->ghist = take<int32_t>(ar, 256 * w->cap_nodes);
    w->tile_node = take<int32_t>(ar, w->cap_tiles);
    w->super_node = take<int32_t>(ar, w->cap_supers);
    w->tbox = take<float>(ar, 12 * w->cap_tiles);
    w->sbox = take<float>(ar, 12 * w->cap_supers);
    w->ctr = take<LCounters>(ar, 1);
    w->small_items = take<SmallItem>(ar, w->cap_small);
    w->buckets = take<SmallItem>(ar, 4 * w->cap_small);
    w->bcount = take<int32_t>(ar, 16);
    w->large_out = take<ChildOut>(ar, w->cap_nodes);
    w->sort_temp_bytes = sort_temp_bytes(m);
    w->sort_temp = arena_take(ar, w->sort_temp_bytes);
    w->root = take<int32_t>(ar, w->cap_nodes);
    w->lhist = take<int32_t>(ar, 16 * w->cap_nodes);
    w->lfeat = take<float>(ar, RS_NFEAT * w->cap_nodes);
    w->lnl = take<float>(ar, w->cap_nodes);
    w->lcnt = take<int32_t>(ar, 2 * w->cap_nodes);
    w->lstat = take<int32_t>(ar, 16);
    w->model = nullptr;
    w->tb.cap_entry = 0;
    return (w->sort_temp && w->lstat) ? RS_OK : RS_EINTERNAL;
}

// Entries: one per child cell record and per leaf (leaves hold up to 64
// members, about 50 on average); the estimate below is several times the
// usual count and grows on overflow.
int tree_reserve(LargeWork* w, int64_t m, int64_t nv, int64_t grow) {
    int64_t cap_inode = (m / 64 + 2 * nv + 1024) * grow;
    int64_t cap_entry = (m / 12 + 64 * nv + 4096) * grow;
    // test hook: a small first capacity exercises the overflow and rebuild path
    if (const char* e = getenv("RS_DEBUG_TREE_ENTRIES")) {
        const int64_t v = atoll(e) * grow;
        if (v > 0 && v < cap_entry) cap_entry = v;
    }
    if (cap_inode > 0x7fffffffll) cap_inode = 0x7fffffffll;
    if (cap_entry > 0x7fffffffll) cap_entry = 0x7fffffffll;
    size_t b = 0;
    auto add = [&](size_t x) { b += arena_round(x); };
    for (int k = 0; k < 5; k++) add(4 * cap_inode);
    for (int k = 0; k < 3; k++) add(4 * cap_entry);
    add(4 * 16 * cap_entry); add(4 * m); add(64);
    Arena* ar;
    RS_TRY(arena_reserve(AR_TREE, b + 4096, &ar));
    TreeBuf& tb = w->tb;
    tb.istart = take<int32_t>(ar, cap_inode);
    tb.iend = take<int32_t>(ar, cap_inode);
    tb.ientry = take<int32_t>(ar, cap_inode);
    tb.cfirst = take<int32_t>(ar, cap_inode);
    tb.ccount = take<int32_t>(ar, cap_inode);
    tb.estart = take<int32_t>(ar, cap_entry);
    tb.eend = take<int32_t>(ar, cap_entry);
    tb.enode = take<int32_t>(ar, cap_entry);
    tb.erec = take<float>(ar, 16 * cap_entry);
    tb.leaf_of = take<int32_t>(ar, m);
    int32_t* ctr = take<int32_t>(ar, 16);
    if (!ctr) return RS_EINTERNAL;
    tb.n_inode = ctr;
    tb.n_entry = ctr + 1;
    tb.overflow = ctr + 2;
    tb.cap_inode = (int32_t)cap_inode;
    tb.cap_entry = (int32_t)cap_entry;
    return RS_OK;
}

// Launches the small-subtree kernels over a device list of small items whose
// members live in `mb`.
int launch_small_items(LargeWork* w, const SmallItem* items, int n, const Members& mb,
                       const NodeRec& nr, const PhaseParams& pp, int32_t* deepest,
                       hipStream_t st) {
    if (n <= 0) return RS_OK;
    RS_HIP(hipMemsetAsync(w->bcount, 0, 16 * sizeof(int32_t), st));
    k_bucket<<<grid_for(n, 256, 1ll << 31), 256, 0, st>>>(items, n, w->buckets, w->cap_small,
                                                          w->bcount);
    RS_HIP(hipGetLastError());
    int32_t* hb = nullptr;
    RS_TRY(host_scratch((void**)&hb, 64));
    RS_HIP(hipMemcpyAsync(hb, w->bcount, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    int cnts[4] = {hb[0], hb[1], hb[2], hb[3]};
    hipStream_t ls = st;
    if (w->side) {
        // on the side stream, after everything the caller's stream queued
        RS_HIP(hipEventRecord(w->side_ready, st));
        RS_HIP(hipStreamWaitEvent(w->side, w->side_ready, 0));
        ls = w->side;
    }
    for (int b = 3; b >= 0; b--)
        RS_TRY(run_small_bucket(b, w->buckets + b * w->cap_small, cnts[b], mb, nr, pp, deepest, ls,
                                w->side ? "phase_small_children" : "phase_small"));
    if (w->side) {
        RS_HIP(hipEventRecord(w->side_done, w->side));
        w->side_pending = true;
    }
    return RS_OK;
}

// the last node whose first index (field F, ascending over the nodes) is at
// most i
template <int32_t LNode::*F>
RS_DEV int32_t node_of(const LNode* __restrict__ nodes, int32_t nv, int32_t i) {
    int32_t lo = 0, hi = nv - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (nodes[mid].*F <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// the level's tile -> node and super-tile -> node maps and its (node, chunk)
// work items of up to LCHUNK members, built from the node table
constexpr int32_t LCHUNK = 4096;

__global__ void k_lmaps(int32_t nv, const LNode* __restrict__ nodes, int32_t tiles,
                        int32_t supers, int32_t ni, int32_t* __restrict__ tile_node,
                        int32_t* __restrict__ super_node, LItem* __restrict__ items) {
    const int32_t n = max(tiles, max(supers, ni));
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += gridDim.x * blockDim.x) {
        if (i < tiles) tile_node[i] = node_of<&LNode::tile0>(nodes, nv, i);
        if (i < supers) super_node[i] = node_of<&LNode::super0>(nodes, nv, i);
        if (i < ni) {
            const int32_t v = node_of<&LNode::item0>(nodes, nv, i);
            const LNode nd = nodes[v];
            const int64_t c = (int64_t)(i - nd.item0) * LCHUNK;
            const int32_t len = (int32_t)min((int64_t)LCHUNK, (int64_t)nd.size - c);
            items[i] = LItem{v, len, nd.in_off + c, nd.t_off + c};
        }
    }
}

// One level over the large nodes `hn` (host copies) whose members live in
// `in`.  Appends the next level's large nodes to `next` (offsets into w->SN).
int large_level(LargeWork* w, const std::vector<ChildOut>& hn, const Members& in,
                const float* X, const float* Y, const float* Z, const PhaseParams& pp,
                const NodeRec& nr, int32_t* deepest, std::vector<ChildOut>* next,
                int64_t* n_accepted, int64_t* n_fallback, hipStream_t st) {
    const int nv = (int)hn.size();
    std::vector<LNode> nodes(nv);
    int64_t toff = 0;
    int32_t tiles = 0, supers = 0, ni = 0;
    for (int v = 0; v < nv; v++) {
        LNode& nd = nodes[v];
        nd.slot = hn[v].slot;
        nd.size = hn[v].size;
        nd.minidx = hn[v].minidx;
        nd.level = hn[v].level;
        nd.in_off = hn[v].off;
        nd.t_off = toff;
        nd.ntile = (nd.size + 63) / 64;
        nd.nsuper = (nd.ntile + 63) / 64;
        nd.nitem = (int32_t)((nd.size + LCHUNK - 1) / LCHUNK);
        nd.tile0 = tiles;
        nd.super0 = supers;
        nd.item0 = ni;
        tiles += nd.ntile;
        supers += nd.nsuper;
        ni += nd.nitem;
        toff += nd.size;
    }
    const int64_t M = toff;
    if (nv > w->cap_nodes || ni > w->cap_items || tiles > w->cap_tiles ||
        supers > w->cap_supers || M > w->cap_m)
        return RS_EINTERNAL;
    RS_HIP(hipMemcpyAsync(w->nodes, nodes.data(), sizeof(LNode) * nv, hipMemcpyHostToDevice, st));
    {
        const int32_t nmap = std::max(tiles, std::max(supers, ni));
        k_lmaps<<<grid_for(nmap, 256), 256, 0, st>>>(nv, w->nodes, tiles, supers, ni,
                                                     w->tile_node, w->super_node, w->items);
        RS_HIP(hipGetLastError());
    }
    RS_HIP(hipMemsetAsync(w->gacc, 0, 8 * 18 * (size_t)nv, st));
    k_lext_init<<<grid_for(6 * nv, 256), 256, 0, st>>>(nv, w->gext);
    const int BT = 256;
    unsigned gm = grid_for(M, BT, 1ll << 31);
    k_lmom<<<ni, 256, 0, st>>>(w->items, w->nodes, in, X, Y, Z, pp, w->gacc, w->gext);
    k_lnorm<<<grid_for(nv, 64), 64, 0, st>>>(nv, w->nodes, w->gacc, w->gext, X, Y, Z, pp, nr,
                                             w->prm);
    k_lkeys<<<ni, 256, 0, st>>>(w->items, in, w->prm, pp, w->kin, w->src, w->lrec);
    RS_HIP(hipGetLastError());
    int vbits = 1;
    while ((1 << vbits) < nv) vbits++;
    RS_TRY(sort_pairs_u64_i32(w->kin, w->kout, w->src, w->perm, M, 42 + vbits, w->sort_temp,
                              w->sort_temp_bytes, st));
    k_lgather<<<gm, BT, 0, st>>>(M, w->perm, w->kout, w->lrec, w->T, w->mnode);
    k_ltbox<<<tiles, 64, 0, st>>>(w->tile_node, w->nodes, w->T, w->prm, pp, w->tbox);
    k_lsbox<<<supers, 64, 0, st>>>(w->super_node, w->nodes, w->tbox, w->sbox);
    k_lcull<<<grid_for(nv, 64), 64, 0, st>>>(nv, w->nodes, w->sbox, pp, w->prm);
    RS_HIP(hipGetLastError());
    std::vector<int32_t> tree_levels;
    // search tree; its buffers grow and the build is redone on overflow
    if (w->tb.cap_entry == 0) RS_TRY(tree_reserve(w, w->cap_m, w->cap_nodes, 1));
    int32_t n_entry = 0;
    for (int64_t grow = 2;; grow *= 2) {
        bool tree_overflow = false;
        RS_TRY(tree_build(w->tb, w->root, w->kout, w->nodes, nv, w->T, w->mnode, w->prm, pp,
                          &tree_levels, &tree_overflow, &n_entry, st));
        if (!tree_overflow) break;
        if (grow > 1024) return RS_EINTERNAL;
        RS_TRY(tree_reserve(w, w->cap_m, w->cap_nodes, grow));
    }
    TArgs TA{w->mnode, w->tile_node, w->nodes, w->prm, w->root, w->tb, w->T, pp,
             M};
    // proposer features (when requested or when a proposal is wanted)
    const bool learned = w->model != nullptr;
    if (pp.want_feat || learned) {
        RS_HIP(hipMemsetAsync(w->lhist, 0, 4 * 16 * (size_t)nv, st));
        k_lfeat<<<ni, 256, 0, st>>>(w->items, in, w->prm, pp, w->lhist);
        k_lfeat_fin<<<grid_for(nv, 64), 64, 0, st>>>(nv, w->nodes, w->gacc, w->lhist, w->lfeat,
                                                    nr, pp.want_feat);
        RS_HIP(hipGetLastError());
    }
    if (learned) {
        RS_TRY(mlp_infer(w->model, nv, w->lfeat, w->lnl, st));
        k_lbracket<<<grid_for(nv, 64), 64, 0, st>>>(nv, w->lnl, w->prm);
        RS_HIP(hipGetLastError());
    }
    prof_begin("phase_large_nn", st);
    RS_TRY(tree_nn(TA, tiles, w->d2, st));
    prof_end("phase_large_nn", st, (double)M);
    if (learned) {
        // exact acceptance of each bracket; rejected nodes are searched again
        RS_HIP(hipMemsetAsync(w->lcnt, 0, 4 * 2 * (size_t)nv, st));
        RS_HIP(hipMemsetAsync(w->lstat, 0, 4 * 4, st));
        k_lcount<<<ni, 256, 0, st>>>(w->items, w->d2, w->prm, w->lcnt);
        k_laccept<<<grid_for(nv, 64), 64, 0, st>>>(nv, w->lcnt, w->prm, w->lstat);
        RS_HIP(hipGetLastError());
        int32_t* hs = nullptr;
        RS_TRY(host_scratch((void**)&hs, 64));
        RS_HIP(hipMemcpyAsync(hs, w->lstat, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        RS_HIP(hipStreamSynchronize(st));
        *n_accepted += hs[0];
        *n_fallback += hs[1];
        if (hs[1] > 0) {
            prof_begin("phase_large_nn_fallback", st);
            RS_TRY(tree_nn(TA, tiles, w->d2, st));
            // the first step's counts, from zero (the bracket's are spent)
            RS_HIP(hipMemsetAsync(w->lcnt, 0, 4 * 2 * (size_t)nv, st));
            k_lcount_refine<<<ni, 256, 0, st>>>(w->items, w->d2, w->prm, w->lcnt);
            k_laccept_refine<<<grid_for(nv, 64), 64, 0, st>>>(nv, w->lcnt, w->prm, w->lstat);
            RS_HIP(hipGetLastError());
            RS_HIP(hipMemcpyAsync(hs + 2, w->lstat + 2, sizeof(int32_t), hipMemcpyDeviceToHost,
                                  st));
            RS_HIP(hipStreamSynchronize(st));
            if (hs[2] > 0) RS_TRY(tree_nn(TA, tiles, w->d2, st));
            prof_end("phase_large_nn_fallback", st, (double)M);
        }
    }
    for (int pass = 0; pass < 4; pass++) {
        int shift = 24 - 8 * pass;
        RS_HIP(hipMemsetAsync(w->ghist, 0, 4 * 256 * (size_t)nv, st));
        k_lhist<<<ni, 256, 0, st>>>(w->items, w->d2, w->prm, shift, w->ghist);
        k_lpick<<<nv, 64, 0, st>>>(w->ghist, shift, w->prm, w->nodes, nr, pass == 3);
        RS_HIP(hipGetLastError());
    }
    k_liota<<<gm, BT, 0, st>>>(M, w->par);
    // only members with d_i^2 <= l^2 can link: shrink the boxes to them
    RS_TRY(tree_refit_active(w->tb, n_entry, tree_levels, w->T, w->mnode, w->prm, pp, w->d2, st));
    prof_begin("phase_large_link", st);
    RS_TRY(tile_link(TA, tiles, w->d2, w->par, st));
    prof_end("phase_large_link", st, (double)M);
    k_lflat<<<gm, BT, 0, st>>>(M, w->par, w->cnt, w->mpk);
    k_lstat<<<gm, BT, 0, st>>>(M, w->par, w->T.idx, w->cnt, w->mpk);
    RS_HIP(hipMemsetAsync(w->ctr, 0, sizeof(LCounters), st));
    // the previous level's small children may still read the child buffers
    if (w->side_pending) RS_HIP(hipStreamWaitEvent(st, w->side_done, 0));
    k_lchild<<<gm, BT, 0, st>>>(M, w->par, w->cnt, w->mpk, w->mnode, w->nodes, pp, nr, w->cslot,
                                w->coff, w->cfill, w->cclass, w->ctr, w->small_items,
                                w->large_out, w->cap_m);
    k_lscatter<<<gm, BT, 0, st>>>(M, w->par, w->T, w->cslot, w->coff, w->cfill, w->cclass, w->SN,
                                  w->SN, deepest);
    RS_HIP(hipGetLastError());
    LCounters hc;
    RS_HIP(hipMemcpyAsync(&hc, w->ctr, sizeof(LCounters), hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    RS_TRY(launch_small_items(w, w->small_items, hc.n_small, w->SN, nr, pp, deepest, st));
    next->resize(hc.n_large);
    if (hc.n_large > 0) {
        RS_HIP(hipMemcpyAsync(next->data(), w->large_out, sizeof(ChildOut) * hc.n_large,
                              hipMemcpyDeviceToHost, st));
        RS_HIP(hipStreamSynchronize(st));
    }
    return RS_OK;
}

}  // namespace rs
