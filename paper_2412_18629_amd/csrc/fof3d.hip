// fof3d.hip -- 3D friends-of-friends over one periodic box (the per-process
// FoF pass of the paper's Parallelization section).
//
// Layout and flow (all device-resident, one stream):
//   1. keys:   each particle gets a 64-bit key (coarse cell << 3 | octant).
//              Coarse cells have side >= ll (plus rounding slack), so every
//              linked pair sits in neighbouring cells; octants (half-side
//              sub-cells) have a diagonal below ll, so all particles of one
//              octant are linked without a test (auto-link).
//   2. sort:   key/index radix sort -> cell-sorted order; positions are
//              gathered into sorted SoA arrays (coalesced reads later).
//   3. tables: occupied octants and cells are enumerated by scans.  Cell
//              keys are x-fastest, so the occupied cells of one (y, z) row
//              are a sorted run; a dense row table gives each row's run
//              (when the grid has few rows for the particle count, else the
//              run is found by binary search over all cell keys).
//   4. link:   union-find over octants (one element each, its members
//              being linked already); octant pairs in the 27-cell
//              neighbourhood are tested with early exit on the first linked
//              pair and skipped when already in one component.  Pairs of
//              more than HEAVY_PAIRS member pairs are queued and tested
//              afterwards, one wavefront per pair.  Without auto-link (grids
//              of under three cells per axis, or octants too wide) the
//              union-find runs over slots and every member pair is tested.
//   5. labels: flatten, slot parents from the octant roots, smallest
//              original index per root, scatter to the caller's labels.
#include <algorithm>
#include <cstdlib>

#include "common.h"

namespace rs {

struct Grid3 {
    int64_t nc;        // cells per axis
    double scale;      // nc / E (fp64), E the side of the gridded cube
    double o[3];       // corner of the gridded cube (0 for a periodic box)
    float L, h, ll2;   // periodic box side and half side (periodic grids only)
    int key_bits;
    bool autolink;     // every octant pair closer than ll
    bool octfilter;    // octant offsets of 3 half-cells cannot link (no wrap, or nc >= 3)
};

// where the particles must lie: a periodic box [0, L), or a sub-box whose
// owned particles [0, n_owned) lie in [lo, hi) and ghosts in the shell
// [lo - gw, hi + gw) (bounds of the shell in fp64)
struct Bounds {
    bool periodic;
    int64_t n_owned;
    float lo[3], hi[3];
    double glo[3], ghi[3];
};

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

__global__ void k_keys(const float* __restrict__ x, const float* __restrict__ y,
                       const float* __restrict__ z, int64_t n, Grid3 g, Bounds B,
                       uint64_t* __restrict__ keys, int32_t* __restrict__ idx,
                       int32_t* __restrict__ err) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float p[3] = {x[i], y[i], z[i]};
    int64_t c[3];
    int o[3];
    bool bad = false;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (B.periodic) bad |= !(p[a] >= 0.0f && p[a] < g.L);
        else if (i < B.n_owned) bad |= !(p[a] >= B.lo[a] && p[a] < B.hi[a]);
        else bad |= !((double)p[a] >= B.glo[a] && (double)p[a] < B.ghi[a]);
        double u = ((double)p[a] - g.o[a]) * g.scale;
        int64_t ci = (int64_t)floor(u);
        int64_t oi = (int64_t)floor(2.0 * u) - 2 * ci;
        if (ci >= g.nc) { ci = g.nc - 1; oi = 1; }
        if (ci < 0) { ci = 0; oi = 0; }
        c[a] = ci;
        o[a] = oi < 0 ? 0 : (oi > 1 ? 1 : (int)oi);
    }
    if (bad) {
        atomicOr(err, 1);
        c[0] = c[1] = c[2] = 0;
    }
    uint64_t cell = (uint64_t)((c[2] * g.nc + c[1]) * g.nc + c[0]);
    keys[i] = (cell << 3) | (uint64_t)(o[2] << 2 | o[1] << 1 | o[0]);
    idx[i] = (int32_t)i;
}

// positions interleaved, 12 bytes a particle, so that the gather below
// fetches one record (one or two cache lines) per particle instead of three
// scattered values
__global__ void k_interleave3(int64_t n, const float* __restrict__ x,
                              const float* __restrict__ y, const float* __restrict__ z,
                              float* __restrict__ rec) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    rec[3 * i] = x[i];
    rec[3 * i + 1] = y[i];
    rec[3 * i + 2] = z[i];
}

__global__ void k_gather3(const int32_t* __restrict__ perm, const float* __restrict__ rec,
                          int64_t n, float* __restrict__ sx, float* __restrict__ sy,
                          float* __restrict__ sz) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t i = perm[s];
    sx[s] = rec[3 * i];
    sy[s] = rec[3 * i + 1];
    sz[s] = rec[3 * i + 2];
}

// run-start flags of octants and of cells in the sorted key order
__global__ void k_run_flags(const uint64_t* __restrict__ keys, int64_t n,
                            int32_t* __restrict__ oflag, int32_t* __restrict__ cflag) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint64_t k = keys[s];
    uint64_t p = s ? keys[s - 1] : ~0ull;
    oflag[s] = (s == 0 || k != p) ? 1 : 0;
    cflag[s] = (s == 0 || (k >> 3) != (p >> 3)) ? 1 : 0;
}

__global__ void k_tables(const uint64_t* __restrict__ keys, int64_t n,
                         const int32_t* __restrict__ oflag, const int32_t* __restrict__ oex,
                         const int32_t* __restrict__ cflag, const int32_t* __restrict__ cex,
                         int32_t* __restrict__ oct_start, uint8_t* __restrict__ oct_bits,
                         int32_t* __restrict__ cell_oct, uint64_t* __restrict__ cell_key) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    if (oflag[s]) {
        int32_t o = oex[s];
        oct_start[o] = (int32_t)s;
        oct_bits[o] = (uint8_t)(keys[s] & 7);
        if (cflag[s]) {
            int32_t c = cex[s];
            cell_oct[c] = o;
            cell_key[c] = keys[s] >> 3;
        }
    }
}

__global__ void k_iota(int64_t n, int32_t* __restrict__ v) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s < n) v[s] = (int32_t)s;
}

// first index in [b, e) whose key is >= k (keys ascending)
RS_DEV int32_t lower_bound_u64(const uint64_t* __restrict__ keys, int32_t b, int32_t e,
                               uint64_t k) {
    while (b < e) {
        const int32_t m = b + ((e - b) >> 1);
        if (keys[m] < k) b = m + 1;
        else e = m;
    }
    return b;
}

// row_start[r] = first cell whose row (key / nc) is >= r, for r in [0, rows]
__global__ void k_row_start(const uint64_t* __restrict__ cell_key, int32_t n_cell, int64_t nc,
                            int64_t rows, int32_t* __restrict__ row_start) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r > rows) return;
    row_start[r] = lower_bound_u64(cell_key, 0, n_cell, (uint64_t)r * (uint64_t)nc);
}

struct LinkArgs {
    const int32_t* oct_start;   // [n_oct + 1]
    const uint8_t* oct_bits;    // [n_oct]
    const int32_t* cell_oct;    // [n_cell + 1]
    const uint64_t* cell_key;   // [n_cell], ascending
    const int32_t* row_start;   // [nc^2 + 1], or null: rows found by binary search
    int32_t n_cell;
    const uint64_t* keys;       // sorted keys
    const float *sx, *sy, *sz;  // sorted positions
    int32_t* parent;            // union-find over octants (auto-link) or over slots
    int32_t n_oct;
    Grid3 g;
    int2* heavy;                // deferred octant pairs (auto-link) ...
    int32_t* n_heavy;           // ... their count (may exceed the capacity)
    int32_t cap_heavy;
};

// octant pairs with more member pairs than this are deferred to a second
// pass, run one wavefront per pair once every lighter pair has been linked:
// by then most of them already share a root, and the rest are searched 64
// member pairs at a time instead of serially by one thread
constexpr int64_t HEAVY_PAIRS = 1024;

// cells of row rr (cell indices [b, e))
RS_DEV void row_cells(const LinkArgs& A, uint64_t rr, int32_t& b, int32_t& e) {
    if (A.row_start) {
        b = A.row_start[rr];
        e = A.row_start[rr + 1];
    } else {
        const uint64_t nc = (uint64_t)A.g.nc;
        b = lower_bound_u64(A.cell_key, 0, A.n_cell, rr * nc);
        e = lower_bound_u64(A.cell_key, b, A.n_cell, (rr + 1) * nc);
    }
}

// pair distance with the periodic shift (PER) or without (sub-box)
template <bool PER>
RS_DEV float link_d2(float xi, float yi, float zi, float xj, float yj, float zj,
                     const Grid3& g) {
    return PER ? pos_d2_wrap(xi, yi, zi, xj, yj, zj, g.L, g.h)
               : pos_d2_nowrap(xi, yi, zi, xj, yj, zj);
}

// test octant a (slots [s0, s1), octant bits oa) against every later octant
// of cell c, which sits at offset (dx, dy, dz) cells from a's cell.
// `ra` is an element of a's component (its last known root): finding from it
// is a short walk; it is brought up to date once per batch of octants and
// after each union (a stale one only costs a redundant test).  With
// auto-link the union-find runs over octant indices (one element per octant,
// a dense array half the size of the slot array); otherwise over slots.
// The auto-linked pass takes the cell's octants in pairs: their octant bits
// and union-find parents are loaded together, so that the latencies overlap
// instead of adding up along the thread's serial walk (the walk is bound by
// them; larger batches spill registers).
constexpr int LINK_BATCH = 2;

// member-pair tests of the counting build (instrumentation level 2)
__device__ unsigned long long g_3d_pairs[64];

template <bool AUTOLINK, bool PER, bool CNT>
RS_DEV void link_cell(const LinkArgs& A, int32_t a, int32_t s0, int32_t s1, int oa, int32_t c,
                      int dx, int dy, int dz, int32_t& ra, unsigned long long& npairs) {
    const Grid3& g = A.g;
    const int32_t b0 = A.cell_oct[c], b1 = A.cell_oct[c + 1];
    // an octant pair is skipped when the filter puts it beyond reach
    auto far = [&](int ob) {
        const int ddx = 2 * dx + (ob & 1) - (oa & 1);
        const int ddy = 2 * dy + ((ob >> 1) & 1) - ((oa >> 1) & 1);
        const int ddz = 2 * dz + (ob >> 2) - (oa >> 2);
        return ddx == 3 || ddx == -3 || ddy == 3 || ddy == -3 || ddz == 3 || ddz == -3;
    };
    if (!AUTOLINK) {
        for (int32_t b = b0 < a + 1 ? a + 1 : b0; b < b1; b++) {
            if (g.octfilter && far(A.oct_bits[b])) continue;
            const int32_t t0 = A.oct_start[b], t1 = A.oct_start[b + 1];
            if (CNT) npairs += (unsigned long long)(s1 - s0) * (unsigned long long)(t1 - t0);
            for (int32_t i = s0; i < s1; i++) {
                const float xi = A.sx[i], yi = A.sy[i], zi = A.sz[i];
                for (int32_t j = t0; j < t1; j++)
                    if (link_d2<PER>(xi, yi, zi, A.sx[j], A.sy[j], A.sz[j], g) <= g.ll2)
                        uf_unite(A.parent, i, j);
            }
        }
        return;
    }
    // every octant is one element: its members are linked already
    for (int32_t base = b0 < a + 1 ? a + 1 : b0; base < b1; base += LINK_BATCH) {
        int obk[LINK_BATCH];
        int32_t pbk[LINK_BATCH];
#pragma unroll
        for (int k = 0; k < LINK_BATCH; k++) {
            const int32_t b = base + k;
            obk[k] = b < b1 ? A.oct_bits[b] : 0;
            pbk[k] = b < b1 ? uf_load(A.parent, b) : 0;
        }
        ra = uf_find(A.parent, ra);
#pragma unroll
        for (int k = 0; k < LINK_BATCH; k++) {
            const int32_t b = base + k;
            if (b >= b1) break;
            if (g.octfilter && far(obk[k])) continue;
            // b hangs below a's root already, or its root is found from the
            // parent loaded above (parents only move up) and stored as b's
            // parent, so that the next octant to meet b reaches it at once
            if (pbk[k] == ra) continue;
            const int32_t rb = pbk[k] == b ? b : uf_find(A.parent, pbk[k]);
            if (rb != pbk[k] && rb != b)
                __hip_atomic_store(A.parent + b, rb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ra == rb) continue;
            const int32_t t0 = A.oct_start[b], t1 = A.oct_start[b + 1];
            if ((int64_t)(s1 - s0) * (t1 - t0) > HEAVY_PAIRS) {
                const int32_t q = atomicAdd(A.n_heavy, 1);
                if (q < A.cap_heavy) {
                    A.heavy[q] = make_int2(a, b);
                    continue;
                }
            }
            bool hit = false;
            for (int32_t i = s0; i < s1 && !hit; i++) {
                const float xi = A.sx[i], yi = A.sy[i], zi = A.sz[i];
                for (int32_t j = t0; j < t1; j++) {
                    if (CNT) npairs++;
                    if (link_d2<PER>(xi, yi, zi, A.sx[j], A.sy[j], A.sz[j], g) <= g.ll2) {
                        hit = true;
                        break;
                    }
                }
            }
            if (hit) {
                uf_unite(A.parent, ra, rb);
                ra = uf_find(A.parent, ra);
            }
        }
    }
}

// one thread per octant: test it against every later octant in the
// 27-cell neighbourhood.  Octants are numbered in cell-key order, so cells
// with a smaller key (among them every cell of an earlier row) hold only
// earlier octants, whose pairs with this one are taken from their side.
template <bool AUTOLINK, bool PER, bool CNT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) k_link(LinkArgs A) {
    const int32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= A.n_oct) return;
    unsigned long long npairs = 0;   // counting build only
    const Grid3& g = A.g;
    const int32_t s0 = A.oct_start[a], s1 = A.oct_start[a + 1];
    const uint64_t cell = A.keys[s0] >> 3;
    const int oa = A.oct_bits[a];
    const int64_t nc = g.nc;
    const int64_t cx = (int64_t)(cell % (uint64_t)nc);
    const uint64_t row = cell / (uint64_t)nc;
    const int64_t cy = (int64_t)(row % (uint64_t)nc);
    const int64_t cz = (int64_t)(row / (uint64_t)nc);

    if (!AUTOLINK) {
        if (CNT) npairs += (unsigned long long)(s1 - s0) * (unsigned long long)(s1 - s0 - 1) / 2;
        for (int32_t i = s0; i < s1; i++) {
            const float xi = A.sx[i], yi = A.sy[i], zi = A.sz[i];
            for (int32_t j = i + 1; j < s1; j++)
                if (link_d2<PER>(xi, yi, zi, A.sx[j], A.sy[j], A.sz[j], g) <= g.ll2)
                    uf_unite(A.parent, i, j);
        }
    }
    int32_t ra = AUTOLINK ? a : s0;
    // x - 1 .. x + 1 are one contiguous key range unless x wraps
    const bool inner = nc >= 3 && cx >= 1 && cx <= nc - 2;
    for (int dz = -1; dz <= 1; dz++) {
        int64_t nz = cz + dz;
        if (!PER && (nz < 0 || nz >= nc)) continue;
        nz = nz < 0 ? nz + nc : (nz >= nc ? nz - nc : nz);
        for (int dy = -1; dy <= 1; dy++) {
            int64_t ny = cy + dy;
            if (!PER && (ny < 0 || ny >= nc)) continue;
            ny = ny < 0 ? ny + nc : (ny >= nc ? ny - nc : ny);
            const uint64_t rr = (uint64_t)(nz * nc + ny);
            if (rr < row) continue;
            int32_t rb, re;
            row_cells(A, rr, rb, re);
            if (rb >= re) continue;
            const uint64_t rbase = rr * (uint64_t)nc;
            if (inner) {
                const uint64_t klo = rbase + (uint64_t)(cx - 1), khi = klo + 2;
                for (int32_t c = lower_bound_u64(A.cell_key, rb, re, klo); c < re; c++) {
                    const uint64_t nkey = A.cell_key[c];
                    if (nkey > khi) break;
                    if (nkey < cell) continue;
                    link_cell<AUTOLINK, PER, CNT>(A, a, s0, s1, oa, c, (int)(nkey - klo) - 1,
                                                  dy, dz, ra, npairs);
                }
            } else {
                for (int dx = -1; dx <= 1; dx++) {
                    int64_t nx = cx + dx;
                    if (!PER && (nx < 0 || nx >= nc)) continue;
                    nx = nx < 0 ? nx + nc : (nx >= nc ? nx - nc : nx);
                    const uint64_t nkey = rbase + (uint64_t)nx;
                    if (nkey < cell) continue;
                    const int32_t c = lower_bound_u64(A.cell_key, rb, re, nkey);
                    if (c < re && A.cell_key[c] == nkey)
                        link_cell<AUTOLINK, PER, CNT>(A, a, s0, s1, oa, c, dx, dy, dz, ra,
                                                      npairs);
                }
            }
        }
    }
    if (CNT && npairs) atomicAdd(&g_3d_pairs[threadIdx.x & 63], npairs);
}


// the deferred octant pairs, one wavefront per pair (grid-stride): skipped
// when already in one component, otherwise the member pairs are tested 64
// at a time until the first one within ll
constexpr int HEAVY_BLOCKS = 8192;

template <bool PER, bool CNT>
__global__ void __launch_bounds__(64) k_link_heavy(LinkArgs A) {
    const int lane = threadIdx.x;
    unsigned long long npairs = 0;   // counting build only
    const int32_t nq = min(*A.n_heavy, A.cap_heavy);
    const Grid3& g = A.g;
    for (int32_t q = blockIdx.x; q < nq; q += gridDim.x) {
        const int2 pr = A.heavy[q];
        const int32_t ra = uf_find(A.parent, pr.x), rb = uf_find(A.parent, pr.y);
        if (__builtin_amdgcn_readfirstlane(ra) == __builtin_amdgcn_readfirstlane(rb)) continue;
        const int32_t s0 = A.oct_start[pr.x], s1 = A.oct_start[pr.x + 1];
        const int32_t t0 = A.oct_start[pr.y], t1 = A.oct_start[pr.y + 1];
        bool hit = false;
        for (int32_t i = s0; i < s1 && !hit; i++) {
            const float xi = A.sx[i], yi = A.sy[i], zi = A.sz[i];
            for (int32_t j0 = t0; j0 < t1 && !hit; j0 += 64) {
                const int32_t j = j0 + lane;
                const bool near = j < t1 && link_d2<PER>(xi, yi, zi, A.sx[j], A.sy[j],
                                                         A.sz[j], g) <= g.ll2;
                if (CNT) npairs += (unsigned long long)min(64, t1 - j0);
                hit = __ballot(near) != 0;
            }
        }
        if (hit && lane == 0) uf_unite(A.parent, ra, rb);
    }
    if (CNT && lane == 0 && npairs) atomicAdd(&g_3d_pairs[blockIdx.x & 63], npairs);
}

// slot parents from the flattened octant roots: each slot points at the
// first slot of its component's root octant (one slot per component is its
// own parent, as with the slot-level union-find)
__global__ void k_oct2slot(int64_t n, const int32_t* __restrict__ oflag,
                           const int32_t* __restrict__ oex, const int32_t* __restrict__ oct_start,
                           const int32_t* __restrict__ poct, int32_t* __restrict__ parent) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t o = oex[s] + oflag[s] - 1;
    parent[s] = oct_start[poct[o]];
}

__global__ void k_flatten(int64_t n, int32_t* __restrict__ parent) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    parent[s] = uf_root(parent, (int)s);
}

// smallest original index per root; sorted slots of one group are mostly
// adjacent, so lanes sharing a root combine before the atomic
__global__ void k_min_index(int64_t n, const int32_t* __restrict__ parent,
                            const int32_t* __restrict__ perm, int32_t* __restrict__ minidx) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool active = s < n;
    const int32_t r = active ? parent[s] : -1;
    const unsigned long long key = active ? (unsigned long long)(uint32_t)perm[s] : ~0ull;
    uint64_t todo = __ballot(active);
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int32_t lr = __shfl(r, leader, 64);
        const bool mine = active && r == lr;
        const uint64_t grp = __ballot(mine);
        // a root held by one lane only needs no reduction
        const unsigned long long mn =
            __popcll(grp) == 1 ? key : wave_min_u64(mine ? key : ~0ull);
        if ((int)(threadIdx.x & 63) == leader) atomicMin(minidx + lr, (int32_t)mn);
        todo &= ~grp;
    }
}

// labels in the caller's order; roots counted per thread over a grid-stride
// loop and reduced per block, so the group counter takes one atomic per
// block rather than one per wavefront
constexpr int WL_BLOCKS = 4096;

__global__ void __launch_bounds__(256)
k_write_labels(int64_t n, const int32_t* __restrict__ parent, const int32_t* __restrict__ perm,
               const int32_t* __restrict__ minidx, int32_t* __restrict__ labels,
               unsigned long long* __restrict__ nroots) {
    __shared__ unsigned long long part[4];
    unsigned long long mine = 0;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = parent[s];
        labels[perm[s]] = minidx[r];
        mine += r == (int32_t)s;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mine += (unsigned long long)__shfl_xor((long long)mine, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long b = part[0] + part[1] + part[2] + part[3];
        if (b) atomicAdd(nroots, b);
    }
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------

// Cell grid over the cube of side E with corner o: cells of side at least
// ll (1 + 2^-20) + E 2^-22, so every pair whose computed D <= ll^2 lies in
// neighbouring cells (the relative term covers the rounding of an unshifted
// difference; across a periodic face the computed difference is never below
// either particle's distance to the face; the absolute term is slack).
static int plan_grid(double E, float ll, bool periodic, const double o[3], float L, Grid3* g) {
    double side_min = (double)ll * (1.0 + ldexp(1.0, -20)) + E * ldexp(1.0, -22);
    int64_t nc = (int64_t)floor(E / side_min);
    if (nc < 1) nc = 1;
    if (nc > (1 << 20)) return RS_EINVAL;
    g->nc = nc;
    g->scale = (double)nc / E;
    for (int a = 0; a < 3; a++) g->o[a] = o[a];
    g->L = L;
    g->h = 0.5f * L;
    g->ll2 = ll * ll;
    double cells = (double)nc * (double)nc * (double)nc;
    int bits = 1;
    while (bits < 61 && ldexp(1.0, bits) < cells) bits++;
    g->key_bits = bits + 3;
    double side = E / (2.0 * (double)nc);
    g->autolink = 3.0 * side * side * (1.0 + 1e-5) <= (double)ll * (double)ll * (1.0 - 1e-5);
    g->octfilter = !periodic || nc >= 3;
    return RS_OK;
}

// dense row table when the grid has few rows for the particle count
static bool use_row_table(int64_t n, const Grid3& g) {
    const uint64_t rows = (uint64_t)g.nc * (uint64_t)g.nc;
    return rows <= std::max<uint64_t>(4 * (uint64_t)n, 1u << 20);
}

// device bytes of one 3D pass (upper bounds: octants and cells <= n)
size_t fof3d_bytes(int64_t n, const Grid3& g) {
    const uint64_t rows = (uint64_t)g.nc * (uint64_t)g.nc;
    size_t bytes = 0;
    auto add = [&](size_t b) { bytes += arena_round(b); };
    add(12 * n);                            // keys and index in; then interleaved positions
    add(8 * n); add(4 * n);                 // keys out, perm
    add(12 * n);                            // sorted positions
    add(4 * n); add(4 * n); add(4 * n); add(4 * n);   // flags + scans
    add(4 * (n + 1)); add(n + 1);           // octant start, bits
    add(4 * (n + 1)); add(8 * (n + 1));     // cell octant start, keys
    add(4 * n); add(4 * n);                 // parent, minidx
    add(4 * (n + 1));                       // octant union-find
    const int64_t cap_heavy = n / 4 + 1024;
    add(8 * cap_heavy); add(64);            // deferred octant pairs, count
    if (use_row_table(n, g)) add(4 * (rows + 1));   // row table
    add(sort_temp_bytes(n)); add(scan_temp_bytes(n));
    add(64);                                // counters
    return bytes;
}

template <bool PER, bool CNT>
static int link_launch(const LinkArgs& A, unsigned go, hipStream_t st) {
    if (A.g.autolink) {
        RS_TRY(fill_i32(A.n_heavy, 0, 1, st));
        k_link<true, PER, CNT><<<go, 256, 0, st>>>(A);
        k_link_heavy<PER, CNT><<<HEAVY_BLOCKS, 64, 0, st>>>(A);
    } else {
        k_link<false, PER, CNT><<<go, 256, 0, st>>>(A);
    }
    RS_HIP(hipGetLastError());
    return RS_OK;
}

template <bool PER>
static int link_pass(const LinkArgs& A, unsigned go, hipStream_t st) {
    if (!prof_count_pairs()) return link_launch<PER, false>(A, go, st);
    // counting build: counters cleared before, read back after (synchronous)
    unsigned long long h[64] = {0};
    RS_HIP(hipStreamSynchronize(st));
    RS_HIP(hipMemcpyToSymbol(HIP_SYMBOL(g_3d_pairs), h, sizeof(h)));
    RS_TRY((link_launch<PER, true>(A, go, st)));
    RS_HIP(hipMemcpyFromSymbolAsync(h, HIP_SYMBOL(g_3d_pairs), sizeof(h), 0,
                                    hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    double sum = 0.0;
    for (int i = 0; i < 64; i++) sum += (double)h[i];
    prof_add_count("pairs_fof3d", sum);
    return RS_OK;
}

// One 3D pass over the work space `ar` (at least fof3d_bytes(n, g), its bump
// pointer at the start); `hcnt` is host memory for 16 counters.  Range
// errors are found before any label is written.
int fof3d_core(const float* x, const float* y, const float* z, int64_t n, const Grid3& g,
               const Bounds& B, Arena* ar, int32_t* hcnt, bool instrument, int32_t* labels,
               int64_t* n_groups, hipStream_t st) {
    const int BT = 256;
    const uint64_t rows = (uint64_t)g.nc * (uint64_t)g.nc;
    const bool row_table = use_row_table(n, g);
    const int64_t cap_heavy = n / 4 + 1024;
    // the sort's keys and indices in share one region, which holds the
    // interleaved positions once the sort has consumed them
    char* kreg = take<char>(ar, 12 * (size_t)n);
    uint64_t* kin = reinterpret_cast<uint64_t*>(kreg);
    int32_t* vin = reinterpret_cast<int32_t*>(kreg + 8 * (size_t)n);
    float* prec = reinterpret_cast<float*>(kreg);
    uint64_t* kout = take<uint64_t>(ar, n);
    int32_t* perm = take<int32_t>(ar, n);
    float* sx = take<float>(ar, n);
    float* sy = take<float>(ar, n);
    float* sz = take<float>(ar, n);
    int32_t* oflag = take<int32_t>(ar, n);
    int32_t* cflag = take<int32_t>(ar, n);
    int32_t* oex = take<int32_t>(ar, n);
    int32_t* cex = take<int32_t>(ar, n);
    int32_t* oct_start = take<int32_t>(ar, n + 1);
    uint8_t* oct_bits = take<uint8_t>(ar, n + 1);
    int32_t* cell_oct = take<int32_t>(ar, n + 1);
    uint64_t* cell_key = take<uint64_t>(ar, n + 1);
    int32_t* parent = take<int32_t>(ar, n);
    int32_t* minidx = take<int32_t>(ar, n);
    int32_t* poct = take<int32_t>(ar, n + 1);
    int2* heavy = take<int2>(ar, cap_heavy);
    int32_t* n_heavy = take<int32_t>(ar, 16);
    int32_t* row_start = row_table ? take<int32_t>(ar, rows + 1) : nullptr;
    size_t stb = sort_temp_bytes(n);
    void* stemp = arena_take(ar, stb);
    void* ctemp = arena_take(ar, scan_temp_bytes(n));
    int32_t* cnt = take<int32_t>(ar, 16);
    if (!cnt) return RS_EINTERNAL;

    unsigned gb = grid_for(n, BT, 1ll << 31);
    RS_TRY(fill_i32(cnt, 0, 16, st));
    k_keys<<<gb, BT, 0, st>>>(x, y, z, n, g, B, kin, vin, cnt + 0);
    RS_HIP(hipGetLastError());
    RS_TRY(sort_pairs_u64_i32(kin, kout, vin, perm, n, g.key_bits, stemp, stb, st));
    k_interleave3<<<gb, BT, 0, st>>>(n, x, y, z, prec);
    k_gather3<<<gb, BT, 0, st>>>(perm, prec, n, sx, sy, sz);
    k_run_flags<<<gb, BT, 0, st>>>(kout, n, oflag, cflag);
    RS_HIP(hipGetLastError());
    RS_TRY(scan_exclusive_i32(oflag, oex, n, ctemp, cnt + 1, st));
    RS_TRY(scan_exclusive_i32(cflag, cex, n, ctemp, cnt + 2, st));
    RS_HIP(hipMemcpyAsync(hcnt, cnt, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    if (hcnt[0]) return RS_ERANGE;
    int32_t n_oct = hcnt[1], n_cell = hcnt[2];

    k_tables<<<gb, BT, 0, st>>>(kout, n, oflag, oex, cflag, cex, oct_start, oct_bits, cell_oct,
                                cell_key);
    RS_HIP(hipGetLastError());
    // sentinels: oct_start[n_oct] = n, cell_oct[n_cell] = n_oct
    RS_TRY(fill_i32(oct_start + n_oct, (int32_t)n, 1, st));
    RS_TRY(fill_i32(cell_oct + n_cell, n_oct, 1, st));
    if (row_table)
        k_row_start<<<grid_for((int64_t)rows + 1, BT, 1ll << 31), BT, 0, st>>>(
            cell_key, n_cell, g.nc, (int64_t)rows, row_start);
    unsigned go = grid_for(n_oct, 256, 1ll << 31);
    if (g.autolink) {
        k_iota<<<go, 256, 0, st>>>(n_oct, poct);
    } else {
        k_iota<<<gb, BT, 0, st>>>(n, parent);
    }
    RS_HIP(hipGetLastError());

    int64_t qcap = std::min<int64_t>(cap_heavy, INT32_MAX);
    // test hook: a smaller queue sends the pairs beyond it down the inline path
    if (const char* e = getenv("RS_DEBUG_HEAVY_QUEUE")) {
        const int64_t v = atoll(e);
        if (v >= 0 && v < qcap) qcap = v;
    }
    LinkArgs A{oct_start, oct_bits, cell_oct, cell_key, row_start, n_cell, kout, sx, sy, sz,
               g.autolink ? poct : parent, n_oct, g, heavy, n_heavy, (int32_t)qcap};
    if (instrument) prof_begin("fof3d_link", st);
    RS_TRY(B.periodic ? link_pass<true>(A, go, st) : link_pass<false>(A, go, st));
    if (instrument) prof_end("fof3d_link", st, (double)n);

    if (g.autolink) {
        k_flatten<<<go, 256, 0, st>>>(n_oct, poct);
        k_oct2slot<<<gb, BT, 0, st>>>(n, oflag, oex, oct_start, poct, parent);
    } else {
        k_flatten<<<gb, BT, 0, st>>>(n, parent);
    }
    RS_TRY(fill_i32(minidx, 0x7fffffff, n, st));
    k_min_index<<<gb, BT, 0, st>>>(n, parent, perm, minidx);
    unsigned long long* nroots = reinterpret_cast<unsigned long long*>(cnt + 4);
    k_write_labels<<<grid_for(n, 256, WL_BLOCKS), 256, 0, st>>>(n, parent, perm, minidx, labels,
                                                               nroots);
    RS_HIP(hipGetLastError());
    unsigned long long* hroots = reinterpret_cast<unsigned long long*>(hcnt + 4);
    RS_HIP(hipMemcpyAsync(hroots, nroots, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    if (n_groups) *n_groups = (int64_t)*hroots;
    return RS_OK;
}

static Bounds periodic_bounds() {
    Bounds B{};
    B.periodic = true;
    return B;
}

int fof3d_plan_periodic(float L, float ll, Grid3* g) {
    const double o[3] = {0.0, 0.0, 0.0};
    return plan_grid((double)L, ll, true, o, L, g);
}

int fof3d_run(const float* x, const float* y, const float* z, int64_t n, float L, float ll,
              int32_t* labels, int64_t* n_groups, hipStream_t st) {
    Grid3 g;
    RS_TRY(fof3d_plan_periodic(L, ll, &g));
    Arena* ar;
    RS_TRY(arena_reserve(AR_BASE, fof3d_bytes(n, g), &ar));
    int32_t* hcnt = nullptr;
    RS_TRY(host_scratch((void**)&hcnt, 64));
    return fof3d_core(x, y, z, n, g, periodic_bounds(), ar, hcnt, true, labels, n_groups, st);
}

// ---------------------------------------------------------------------------
// the 3D pass without allocation: its work space is a fixed device array
// ---------------------------------------------------------------------------

// 128 MiB per device, held from the library's load until the process ends.
// In host code `scratch` names a host-side stand-in, never the device
// memory: the device address comes from hipGetSymbolAddress, once per device.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];
static void* g_scratch_ptr[64];
static int32_t g_noalloc_counts[64][16];   // host counters read back by the pass

int fof3d_noalloc_run(const float* x, const float* y, const float* z, int64_t n, float L,
                      float ll, int32_t* labels, int64_t* n_groups, hipStream_t st) {
    Grid3 g;
    RS_TRY(fof3d_plan_periodic(L, ll, &g));
    if (fof3d_bytes(n, g) > NOALLOC_SCRATCH_BYTES) return RS_EINVAL;
    int dev = 0;
    RS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return RS_EDEVICE;
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return RS_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    Arena a;
    a.base = static_cast<char*>(g_scratch_ptr[dev]);
    a.cap = NOALLOC_SCRATCH_BYTES;
    a.off = 0;
    return fof3d_core(x, y, z, n, g, periodic_bounds(), &a, g_noalloc_counts[dev], false, labels,
                      n_groups, st);
}

// ghost links: (g, label[g]) for the ghosts g >= n_owned whose group holds an
// owned particle, i.e. whose label (the group's smallest index) is < n_owned
__global__ void k_ghost_flag(int64_t n, int64_t n_owned, const int32_t* __restrict__ labels,
                             int32_t* __restrict__ flag) {
    const int64_t g = n_owned + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g < n) flag[g - n_owned] = labels[g] < n_owned ? 1 : 0;
}

__global__ void k_ghost_write(int64_t n, int64_t n_owned, const int32_t* __restrict__ labels,
                              const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                              int32_t* __restrict__ links) {
    const int64_t g = n_owned + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= n || !flag[g - n_owned]) return;
    const int64_t q = pos[g - n_owned];
    links[2 * q] = (int32_t)g;
    links[2 * q + 1] = labels[g];
}

int fof3d_subbox_run(const float* x, const float* y, const float* z, int64_t n,
                     int64_t n_owned, const float* lo, const float* hi, float gw, float ll,
                     int32_t* labels, int32_t* ghost_links, int64_t* n_links, hipStream_t st) {
    Bounds B{};
    B.periodic = false;
    B.n_owned = n_owned;
    double o[3], E = 0.0;
    for (int a = 0; a < 3; a++) {
        B.lo[a] = lo[a];
        B.hi[a] = hi[a];
        B.glo[a] = (double)lo[a] - (double)gw;
        B.ghi[a] = (double)hi[a] + (double)gw;
        o[a] = B.glo[a];
        E = std::max(E, B.ghi[a] - B.glo[a]);
    }
    Grid3 g;
    RS_TRY(plan_grid(E, ll, false, o, 0.0f, &g));
    const int64_t ng = n - n_owned;
    size_t bytes = fof3d_bytes(n, g);
    const bool links = ghost_links != nullptr;
    if (links) bytes += 2 * arena_round(4 * (size_t)(ng + 1)) + arena_round(scan_temp_bytes(ng));
    Arena* ar;
    RS_TRY(arena_reserve(AR_BASE, bytes, &ar));
    int32_t* hcnt = nullptr;
    RS_TRY(host_scratch((void**)&hcnt, 64));
    RS_TRY(fof3d_core(x, y, z, n, g, B, ar, hcnt, true, labels, nullptr, st));
    if (!links) return RS_OK;
    if (ng == 0) {
        *n_links = 0;
        return RS_OK;
    }
    // the 3D pass's work space is done with: its tail holds the link buffers
    int32_t* flag = take<int32_t>(ar, ng + 1);
    int32_t* pos = take<int32_t>(ar, ng + 1);
    void* ctemp = arena_take(ar, scan_temp_bytes(ng));
    if (!ctemp) return RS_EINTERNAL;
    const unsigned gg = grid_for(ng, 256, 1ll << 31);
    k_ghost_flag<<<gg, 256, 0, st>>>(n, n_owned, labels, flag);
    RS_HIP(hipGetLastError());
    RS_TRY(scan_exclusive_i32(flag, pos, ng, ctemp, pos + ng, st));
    k_ghost_write<<<gg, 256, 0, st>>>(n, n_owned, labels, flag, pos, ghost_links);
    RS_HIP(hipGetLastError());
    RS_HIP(hipMemcpyAsync(hcnt, pos + ng, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    *n_links = hcnt[0];
    return RS_OK;
}

}  // namespace rs
