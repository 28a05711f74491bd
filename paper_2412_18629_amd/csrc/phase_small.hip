// phase_small.hip -- whole 6D subtree of a small node inside one workgroup.
//
// A node of at most MAXN members is loaded into LDS once; the workgroup then
// splits it and every descendant without leaving LDS, using an explicit
// stack.  Per node:
//   1. exact integer moments (wave shuffles + LDS atomics) -> a, c
//   2. nearest-neighbour d^2 of every member: every pair once, LDS broadcast
//      reads, R members per thread held in registers, the later member's
//      minimum by a wavefront reduction and an LDS atomic minimum
//   3. l^2 = k-th smallest d^2 by a 4-pass 8-bit radix select in LDS
//   4. links d^2 <= l^2 among members with d^2_i <= l^2 (others cannot link),
//      lock-free union-find in LDS
//   5. components -> children (>= min_sub, not the whole node): node records
//      get global slots, members are regrouped so each child is a contiguous
//      range, children are pushed
// The node's smallest-index member is the moment reference; children carry
// theirs from the packed (index, slot) minimum of their component.
#include <type_traits>

#include "phase_common.h"

namespace rs {

// LDS scalars
enum { SH_SP, SH_S0, SH_SZ, SH_SLOT, SH_LEVEL, SH_REF, SH_NC, SH_NCH, SH_BASE, SH_OK, SH_TOT,
       SH_BUCKET, SH_KK, SH_NOWRAP, SH_N };

// Per member 48 bytes: position and index, velocity and nearest-neighbour
// d^2 (whose slot holds the component counts in step 5), parent, packed
// component minimum, two 16-bit member lists.  At the default min_sub this
// keeps three 1024-member workgroups per CU.
size_t small_lds_bytes(int maxn, int min_sub) {
    int capn = maxn / min_sub + 1;
    return (size_t)maxn * 48 + (size_t)capn * 5 * 4 + (size_t)capn * 6 * 4 + 64;
}

// minimum over the 64 lanes of a non-negative float (or +inf), uniform:
// row steps by DPP, then two row broadcasts carry it to lane 63.  All 64
// lanes must be active.  Rows a broadcast skips read the identity (all
// ones), so each step is one DPP minimum.
RS_DEV float small_wmin_nonneg(float x) {
    uint32_t v = __float_as_uint(x);
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0xB1, 0xf, 0xf, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x4E, 0xf, 0xf, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x124, 0xf, 0xf, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x128, 0xf, 0xf, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x142, 0xa, 0xf, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x143, 0xc, 0xf, false));
    return __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)v, 63));
}

template <int MAXN, int NT, bool FEAT>
__global__ void __launch_bounds__(NT)
k_small_subtree(const SmallItem* __restrict__ items, int n_items, Members mb, NodeRec nr,
                PhaseParams pp, int32_t* __restrict__ deepest) {
    constexpr int R = (MAXN + NT - 1) / NT;
    extern __shared__ __align__(16) char smem[];
    float4* P = reinterpret_cast<float4*>(smem);                  // x y z idx
    float4* V = P + MAXN;                                         // vx vy vz d2
    int32_t* par = reinterpret_cast<int32_t*>(V + MAXN);
    unsigned long long* mpk = reinterpret_cast<unsigned long long*>(par + MAXN);
    uint16_t* perm = reinterpret_cast<uint16_t*>(mpk + MAXN);
    uint16_t* tmp = perm + MAXN;
    const int capn = MAXN / pp.min_sub + 1;
    int32_t* stk = reinterpret_cast<int32_t*>(tmp + MAXN);        // [capn][5]
    int32_t* ch = stk + 5 * capn;                                 // [capn][6]
    __shared__ unsigned long long acc[18];
    __shared__ uint32_t ext[6];
    // the 256-bin histogram of the select (and the feature bins) lives in the
    // member list `tmp` where that is large enough: the two are never live
    // together (steps 1-3 against steps 4-5, separated by barriers)
    constexpr bool HIST_IN_TMP = MAXN >= 512;
    __shared__ int32_t hist_own[HIST_IN_TMP ? 1 : 256];
    int32_t* hist = HIST_IN_TMP ? reinterpret_cast<int32_t*>(tmp) : hist_own;
    __shared__ int32_t sh[SH_N];
    __shared__ float shf[4];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
        const SmallItem it = items[w];
        const int n = it.size;
        if (tid == 0) {
            stk[0] = 0;
            stk[1] = n;
            stk[2] = it.slot;
            stk[3] = it.level;
            stk[4] = 0;
            sh[SH_SP] = 1;
        }
        __syncthreads();
        for (int m = tid; m < n; m += NT) {
            int64_t g = it.off + m;
            P[m] = make_float4(mb.x[g], mb.y[g], mb.z[g], __int_as_float(mb.idx[g]));
            V[m] = make_float4(mb.vx[g], mb.vy[g], mb.vz[g], 0.0f);
            perm[m] = (uint16_t)m;
            if (mb.idx[g] == it.refidx) stk[4] = m;   // exactly one member matches
        }
        __syncthreads();

        for (;;) {
            const int sp_now = sh[SH_SP];
            __syncthreads();                 // every thread has read the stack depth
            if (sp_now == 0) break;
            if (tid == 0) {
                int t = --sh[SH_SP];
                sh[SH_S0] = stk[5 * t + 0];
                sh[SH_SZ] = stk[5 * t + 1];
                sh[SH_SLOT] = stk[5 * t + 2];
                sh[SH_LEVEL] = stk[5 * t + 3];
                sh[SH_REF] = stk[5 * t + 4];
            }
            if (tid < 18) acc[tid] = 0;
            if (tid < 3) ext[tid] = 0xffffffffu;
            else if (tid < 6) ext[tid] = 0u;
            __syncthreads();
            const int s0 = sh[SH_S0], sz = sh[SH_SZ], slot = sh[SH_SLOT], level = sh[SH_LEVEL];
            const int rslot = sh[SH_REF];

            // ---- 1. moments and extents ----
            {
                float4 pr = P[rslot];
                int64_t qref[3] = {quant_pos(pr.x), quant_pos(pr.y), quant_pos(pr.z)};
                Moments mo;
                mom_zero(mo);
                uint32_t mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, mx[3] = {0u, 0u, 0u};
                for (int m = tid; m < sz; m += NT) {
                    int s = perm[s0 + m];
                    float4 p = P[s], v = V[s];
                    mom_add(mo, p.x, p.y, p.z, v.x, v.y, v.z, qref, pp.LQ);
                    uint32_t b[3] = {__float_as_uint(p.x), __float_as_uint(p.y),
                                     __float_as_uint(p.z)};
#pragma unroll
                    for (int ax = 0; ax < 3; ax++) {
                        mn[ax] = b[ax] < mn[ax] ? b[ax] : mn[ax];
                        mx[ax] = b[ax] > mx[ax] ? b[ax] : mx[ax];
                    }
                }
                int active = sz < NT ? sz : NT;
                if (wave * 64 < active) {
                    mom_wave_reduce(mo);
#pragma unroll
                    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
                        for (int ax = 0; ax < 3; ax++) {
                            uint32_t o1 = (uint32_t)__shfl_xor((int)mn[ax], off, 64);
                            uint32_t o2 = (uint32_t)__shfl_xor((int)mx[ax], off, 64);
                            mn[ax] = o1 < mn[ax] ? o1 : mn[ax];
                            mx[ax] = o2 > mx[ax] ? o2 : mx[ax];
                        }
                    }
                    if (lane == 0) {
                        mom_accumulate(acc, mo);
#pragma unroll
                        for (int ax = 0; ax < 3; ax++) {
                            atomicMin(ext + ax, mn[ax]);
                            atomicMax(ext + 3 + ax, mx[ax]);
                        }
                    }
                }
            }
            __syncthreads();
            if (tid == 0) {
                Norm nm = mom_finalize(acc, sz);
                shf[0] = nm.a;
                shf[1] = nm.c;
                shf[2] = nm.sx2;
                shf[3] = nm.sv2;
                bool nowrap = true;
#pragma unroll
                for (int ax = 0; ax < 3; ax++) {
                    float e = __uint_as_float(ext[3 + ax]) - __uint_as_float(ext[ax]);
                    nowrap = nowrap && (e <= pp.h);
                }
                sh[SH_NOWRAP] = nowrap ? 1 : 0;
                nr.a[slot] = nm.a;
                nr.c[slot] = nm.c;
                nr.sx2[slot] = nm.sx2;
                nr.sv2[slot] = nm.sv2;
            }
            __syncthreads();
            const float fa = shf[0], fc = shf[1];
            const bool nowrap = sh[SH_NOWRAP] != 0;

            // ---- proposer features (only when requested) ----
            if (FEAT) {
                if (tid < 16) hist[tid] = 0;
                __syncthreads();
                const float4 pr = P[rslot];
                const FeatFrame fr = feat_frame(acc, sz, pr.x, pr.y, pr.z, shf[2], shf[3]);
                for (int m = tid; m < sz; m += NT) {
                    int s = perm[s0 + m];
                    float4 p = P[s], v = V[s];
                    int br, bv;
                    feat_member_bins(fr, p.x, p.y, p.z, v.x, v.y, v.z, pp.L, pp.h, &br, &bv);
                    atomicAdd(hist + br, 1);
                    atomicAdd(hist + bv, 1);
                }
                __syncthreads();
                if (tid == 0) feat_write(nr.feat + (int64_t)slot * RS_NFEAT, acc, sz, level, hist);
                __syncthreads();
            }

            // ---- 2. nearest-neighbour distances ----
            // Each pair is evaluated once, by the thread holding its earlier
            // member (d^2 is symmetric bit for bit: the differences only
            // change sign).  The later member's minimum is gathered over the
            // wavefront and merged with an LDS atomic minimum on the d^2 bits
            // (non-negative floats order like their bit patterns); a
            // wavefront skips a candidate no member of its row precedes.
            for (int m = tid; m < sz; m += NT) V[perm[s0 + m]].w = __builtin_huge_valf();
            {
                float xi[R], yi[R], zi[R], ui[R], vi[R], wi[R], best[R];
                int si[R];
#pragma unroll
                for (int r = 0; r < R; r++) {
                    int m = tid + r * NT;
                    int s = m < sz ? perm[s0 + m] : perm[s0];
                    si[r] = m < sz ? s : -1;
                    float4 p = P[s], v = V[s];
                    xi[r] = p.x; yi[r] = p.y; zi[r] = p.z;
                    ui[r] = v.x; vi[r] = v.y; wi[r] = v.z;
                    best[r] = __builtin_huge_valf();
                }
                __syncthreads();
                auto scan = [&](auto wrap) {
                    constexpr bool WRAP = decltype(wrap)::value;
                    for (int jj = wave * 64 + 1; jj < sz; jj++) {
                        const int j = perm[s0 + jj];
                        const float4 p = P[j], v = V[j];
                        float rev = __builtin_huge_valf();
#pragma unroll
                        for (int r = 0; r < R; r++) {
                            if (jj > r * NT + wave * 64) {   // uniform over the wavefront
                                const float d = phase_d2<WRAP>(xi[r], yi[r], zi[r], ui[r], vi[r],
                                                               wi[r], p.x, p.y, p.z, v.x, v.y,
                                                               v.z, fa, fc, pp.L, pp.h);
                                const bool ok = tid + r * NT < jj;
                                best[r] = ok && d < best[r] ? d : best[r];
                                rev = ok ? fminf(rev, d) : rev;
                            }
                        }
                        const float mn = small_wmin_nonneg(rev);
                        if (lane == 0 && mn < __builtin_huge_valf())
                            atomicMin(reinterpret_cast<uint32_t*>(&V[j].w), __float_as_uint(mn));
                    }
                };
                if (nowrap) scan(std::false_type{});
                else scan(std::true_type{});
#pragma unroll
                for (int r = 0; r < R; r++)
                    if (si[r] >= 0)
                        atomicMin(reinterpret_cast<uint32_t*>(&V[si[r]].w),
                                  __float_as_uint(best[r]));
            }
            __syncthreads();

            // ---- 3. k-th smallest nearest-neighbour distance ----
            uint32_t prefix = 0, pmask = 0;
            {
                int kk = (int)select_rank(sz, pp.f_ppm);
                for (int pass = 0; pass < 4; pass++) {
                    const int shift = 24 - 8 * pass;
                    for (int b = tid; b < 256; b += NT) hist[b] = 0;
                    __syncthreads();
                    for (int m = tid; m < sz; m += NT) {
                        uint32_t u = __float_as_uint(V[perm[s0 + m]].w);
                        if ((u & pmask) == prefix) atomicAdd(hist + ((u >> shift) & 255u), 1);
                    }
                    __syncthreads();
                    if (wave == 0) {
                        int h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2],
                            h3 = hist[4 * lane + 3];
                        int tot = h0 + h1 + h2 + h3, inc = tot;
#pragma unroll
                        for (int o = 1; o < 64; o <<= 1) {
                            int t = __shfl_up(inc, o, 64);
                            if (lane >= o) inc += t;
                        }
                        int before = inc - tot;
                        if (before < kk && kk <= inc) {
                            int k2 = kk - before, b = 4 * lane;
                            if (k2 > h0) { k2 -= h0; b++;
                                if (k2 > h1) { k2 -= h1; b++;
                                    if (k2 > h2) { k2 -= h2; b++; } } }
                            sh[SH_BUCKET] = b;
                            sh[SH_KK] = k2;
                        }
                    }
                    __syncthreads();
                    prefix |= (uint32_t)sh[SH_BUCKET] << shift;
                    pmask |= 255u << shift;
                    kk = sh[SH_KK];
                }
            }
            const float l2 = __uint_as_float(prefix);

            // ---- 4. links within l ----
            for (int m = tid; m < sz; m += NT) {
                int s = perm[s0 + m];
                par[s] = s;
            }
            if (tid == 0) {
                sh[SH_NC] = 0;
                nr.l2[slot] = l2;
            }
            __syncthreads();
            for (int m = tid; m < sz; m += NT) {
                int s = perm[s0 + m];
                if (V[s].w <= l2) tmp[atomicAdd(sh + SH_NC, 1)] = (uint16_t)s;
            }
            __syncthreads();
            {
                const int nc = sh[SH_NC];
                float xi[R], yi[R], zi[R], ui[R], vi[R], wi[R];
                int si[R];
#pragma unroll
                for (int r = 0; r < R; r++) {
                    int p = tid + r * NT;
                    int s = p < nc ? tmp[p] : 0;
                    si[r] = p < nc ? s : -1;
                    float4 a4 = P[s], b4 = V[s];
                    xi[r] = a4.x; yi[r] = a4.y; zi[r] = a4.z;
                    ui[r] = b4.x; vi[r] = b4.y; wi[r] = b4.z;
                }
                const int q0 = wave * 64 + 1;
                for (int q = q0; q < nc; q++) {
                    int j = tmp[q];
                    float4 p = P[j], v = V[j];
#pragma unroll
                    for (int r = 0; r < R; r++) {
                        int pidx = tid + r * NT;
                        if (si[r] >= 0 && q > pidx) {
                            float d = nowrap
                                ? phase_d2<false>(xi[r], yi[r], zi[r], ui[r], vi[r], wi[r], p.x,
                                                  p.y, p.z, v.x, v.y, v.z, fa, fc, pp.L, pp.h)
                                : phase_d2<true>(xi[r], yi[r], zi[r], ui[r], vi[r], wi[r], p.x,
                                                 p.y, p.z, v.x, v.y, v.z, fa, fc, pp.L, pp.h);
                            if (d <= l2) lds_unite(par, si[r], j);
                        }
                    }
                }
            }
            __syncthreads();

            // ---- 5. components and children ----
            for (int m = tid; m < sz; m += NT) {
                int s = perm[s0 + m];
                par[s] = lds_root(par, s);
                V[s].w = 0.0f;           // component count (exact small integers)
                mpk[s] = ~0ull;
            }
            if (tid == 0) sh[SH_NCH] = 0;
            __syncthreads();
            for (int m = tid; m < sz; m += NT) {
                int s = perm[s0 + m];
                int r = par[s];
                atomicAdd(&V[r].w, 1.0f);
                unsigned long long key =
                    ((unsigned long long)(uint32_t)__float_as_int(P[s].w) << 16) | (unsigned)s;
                atomicMin(mpk + r, key);
            }
            __syncthreads();
            for (int m = tid; m < sz; m += NT) {
                int s = perm[s0 + m];
                const int cs = (int)V[s].w;
                if (par[s] == s && cs >= pp.min_sub && cs < sz) {
                    int c = atomicAdd(sh + SH_NCH, 1);
                    ch[6 * c + 0] = s;
                    ch[6 * c + 1] = cs;
                    ch[6 * c + 2] = (int)(mpk[s] >> 16);
                    ch[6 * c + 3] = (int)(mpk[s] & 0xffffull);
                }
            }
            __syncthreads();
            const int nch = sh[SH_NCH];
            if (nch > 0) {
                if (tid == 0) {
                    int base = atomicAdd(nr.count, nch);
                    bool ok = base + nch <= nr.cap;
                    if (!ok) atomicOr(nr.overflow, 1);
                    sh[SH_OK] = ok ? 1 : 0;
                    sh[SH_BASE] = base;
                    int off = 0;
                    for (int c = 0; c < nch; c++) {
                        ch[6 * c + 4] = off;
                        ch[6 * c + 5] = 0;
                        off += ch[6 * c + 1];
                    }
                    sh[SH_TOT] = off;
                }
                __syncthreads();
                if (sh[SH_OK]) {
                    const int base = sh[SH_BASE];
                    for (int c = tid; c < nch; c += NT) {
                        int cs = base + c;
                        nr.level[cs] = level + 1;
                        nr.minidx[cs] = ch[6 * c + 2];
                        nr.parent[cs] = slot;
                        nr.size[cs] = ch[6 * c + 1];
                        V[ch[6 * c + 0]].w = (float)-(c + 1);
                    }
                    __syncthreads();
                    for (int m = tid; m < sz; m += NT) {
                        int s = perm[s0 + m];
                        int cv = (int)V[par[s]].w;
                        if (cv < 0) {
                            int c = -cv - 1;
                            int pos = ch[6 * c + 4] + atomicAdd(ch + 6 * c + 5, 1);
                            tmp[pos] = (uint16_t)s;
                            deepest[__float_as_int(P[s].w)] = base + c;
                        }
                    }
                    __syncthreads();
                    const int tot = sh[SH_TOT];
                    for (int m = tid; m < tot; m += NT) perm[s0 + m] = tmp[m];
                    if (tid == 0) {
                        int sp = sh[SH_SP];
                        for (int c = 0; c < nch; c++) {
                            int* e = stk + 5 * (sp + c);
                            e[0] = s0 + ch[6 * c + 4];
                            e[1] = ch[6 * c + 1];
                            e[2] = base + c;
                            e[3] = level + 1;
                            e[4] = ch[6 * c + 3];
                        }
                        sh[SH_SP] = sp + nch;
                    }
                }
            }
            __syncthreads();
        }
        __syncthreads();
    }
}

template <int MAXN, int NT>
static int launch_small(const SmallItem* items, int n_items, const Members& mb,
                        const NodeRec& nr, const PhaseParams& pp, int32_t* deepest,
                        hipStream_t st, const char* timer) {
    if (n_items <= 0) return RS_OK;
    size_t lds = small_lds_bytes(MAXN, pp.min_sub);
    auto kern = pp.want_feat ? k_small_subtree<MAXN, NT, true> : k_small_subtree<MAXN, NT, false>;
    RS_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    unsigned grid = (unsigned)(n_items < (1 << 20) ? n_items : (1 << 20));
    prof_begin(timer, st);
    kern<<<grid, NT, lds, st>>>(items, n_items, mb, nr, pp, deepest);
    RS_HIP(hipGetLastError());
    prof_end(timer, st, 0.0);
    return RS_OK;
}

// bucket b: 0 -> <= 64 members, 1 -> <= 256, 2 -> <= 1024, 3 -> <= 2048
int small_bucket_of(int size) { return size <= 64 ? 0 : size <= 256 ? 1 : size <= 1024 ? 2 : 3; }

// Threads per workgroup of buckets 1..3, from the tuning table (each value is
// one of the compiled shapes; results do not depend on the choice).
int run_small_bucket(int b, const SmallItem* items, int n_items, const Members& mb,
                     const NodeRec& nr, const PhaseParams& pp, int32_t* deepest,
                     hipStream_t st, const char* timer) {
    switch (b) {
        case 0: return launch_small<64, 64>(items, n_items, mb, nr, pp, deepest, st, timer);
        case 1:
            if (tune_get(TUNE_SMALL_NT_256) == 128)
                return launch_small<256, 128>(items, n_items, mb, nr, pp, deepest, st, timer);
            return launch_small<256, 256>(items, n_items, mb, nr, pp, deepest, st, timer);
        case 2:
            if (tune_get(TUNE_SMALL_NT_1024) == 256)
                return launch_small<1024, 256>(items, n_items, mb, nr, pp, deepest, st, timer);
            if (tune_get(TUNE_SMALL_NT_1024) == 1024)
                return launch_small<1024, 1024>(items, n_items, mb, nr, pp, deepest, st, timer);
            return launch_small<1024, 512>(items, n_items, mb, nr, pp, deepest, st, timer);
        default:
            if (tune_get(TUNE_SMALL_NT_2048) == 512)
                return launch_small<SMALL_MAX, 512>(items, n_items, mb, nr, pp, deepest, st, timer);
            return launch_small<SMALL_MAX, 1024>(items, n_items, mb, nr, pp, deepest, st, timer);
    }
}

}  // namespace rs
