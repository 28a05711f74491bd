/*
 * fof_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded CPU reference for the two steps the paper
 * names in its Parallelization section: a 3D friends-of-friends pass over one
 * process's periodic sub-box, and, inside every FoF halo, subhalo finding in
 * 6D phase space (Rockstar's hierarchical phase-space FoF, which the paper
 * cites in its Summary for the method).  Only the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg may load this library; the product
 * path never does.  It shares no code with the GPU library.
 *
 * The result is a pure function of the particle set:
 *   3D:  the transitive closure of the pair relation D(i,j) <= ll^2, labels
 *        equal to the smallest member index of each group.
 *   6D:  for each 3D group of at least min_group members (a level-0 node):
 *        dispersions from exact integer moments -> metric factors a, c;
 *        every member's nearest-neighbour distance d_i^2 under
 *        d^2 = a*Dx + c*Dv; the node's linking length l^2 = the k-th smallest
 *        d_i^2 with k = ceil(f n); links d^2(i,j) <= l^2; components of at
 *        least min_sub members (other than the whole node) become children,
 *        which are split again.
 *
 * Floating-point readings (fixed here, identical on the GPU side):
 *   dx = fl(xi - xj), then one periodic image shift:
 *        dx > L/2 -> fl(dx - L);  dx < -L/2 -> fl(dx + L)
 *   D  = fl( fl( fl(dx*dx) + fl(dy*dy) ) + fl(dz*dz) ), no FMA contraction
 *   d^2 = fl( fl(a*Dx) + fl(c*Dv) ), Dv as D over velocity differences
 * Build with -ffp-contract=off -fno-fast-math.
 *
 * Acceleration structures (a 3D cell grid for the FoF pass, a 6D k-d tree
 * inside nodes) only restrict which pairs are evaluated; pruning uses lower
 * bounds with a wide safety margin, and the brute-force paths (all pairs)
 * are kept and selectable for pinning.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

/* ------------------------------------------------------------------ */
/* pair arithmetic                                                     */
/* ------------------------------------------------------------------ */

static float min_image(float d, float L, float h)
{
    if (d > h) return d - L;
    if (d < -h) return d + L;
    return d;
}

static float pos_d2(const float *x, const float *y, const float *z,
                    int64_t i, int64_t j, float L, float h)
{
    float dx = min_image(x[i] - x[j], L, h);
    float dy = min_image(y[i] - y[j], L, h);
    float dz = min_image(z[i] - z[j], L, h);
    float sx = dx * dx, sy = dy * dy, sz = dz * dz;
    float t = sx + sy;
    return t + sz;
}

static float vel_d2(const float *vx, const float *vy, const float *vz,
                    int64_t i, int64_t j)
{
    float dx = vx[i] - vx[j], dy = vy[i] - vy[j], dz = vz[i] - vz[j];
    float sx = dx * dx, sy = dy * dy, sz = dz * dz;
    float t = sx + sy;
    return t + sz;
}

typedef struct {
    const float *x, *y, *z, *vx, *vy, *vz;
    float L, h;
} parts_t;

static float phase_d2(const parts_t *p, int64_t i, int64_t j, float a, float c)
{
    float Dx = pos_d2(p->x, p->y, p->z, i, j, p->L, p->h);
    float Dv = vel_d2(p->vx, p->vy, p->vz, i, j);
    float u = a * Dx, w = c * Dv;
    return u + w;
}

/* ------------------------------------------------------------------ */
/* union-find whose root is always the smallest element                */
/* ------------------------------------------------------------------ */

static int64_t uf_find(int64_t *parent, int64_t i)
{
    while (parent[i] != i) {
        parent[i] = parent[parent[i]];
        i = parent[i];
    }
    return i;
}

static void uf_union(int64_t *parent, int64_t a, int64_t b)
{
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a < b) parent[b] = a; else parent[a] = b;
}

/* ------------------------------------------------------------------ */
/* 3D FoF                                                              */
/* ------------------------------------------------------------------ */

static int check_positions(const float *x, const float *y, const float *z,
                           int64_t n, float L)
{
    for (int64_t i = 0; i < n; i++) {
        if (!(x[i] >= 0.0f && x[i] < L)) return -2;
        if (!(y[i] >= 0.0f && y[i] < L)) return -2;
        if (!(z[i] >= 0.0f && z[i] < L)) return -2;
    }
    return 0;
}

/* All pairs.  O(n^2); reference for the grid version and for tiny boxes. */
int oracle_fof3d_brute(const float *x, const float *y, const float *z,
                       int64_t n, float L, float ll, int32_t *labels)
{
    if (n < 0 || !(L > 0.0f) || !(ll > 0.0f)) return -1;
    if (check_positions(x, y, z, n, L)) return -2;
    float h = 0.5f * L, ll2 = ll * ll;
    int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!parent) return -3;
    for (int64_t i = 0; i < n; i++) parent[i] = i;
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = i + 1; j < n; j++)
            if (pos_d2(x, y, z, i, j, L, h) <= ll2) uf_union(parent, i, j);
    for (int64_t i = 0; i < n; i++) labels[i] = (int32_t)uf_find(parent, i);
    free(parent);
    return 0;
}

typedef struct { int64_t key, idx; } kv_t;

static int cmp_kv(const void *pa, const void *pb)
{
    const kv_t *a = (const kv_t *)pa, *b = (const kv_t *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->idx < b->idx ? -1 : (a->idx > b->idx);
}

/* first position in sorted[0..m) with key >= k */
static int64_t lower_key(const kv_t *s, int64_t m, int64_t k)
{
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (s[mid].key < k) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/*
 * Periodic cell grid of nc^3 cells whose side L/nc is at least
 * ll (1 + 2^-20) + L 2^-22.  A pair whose computed D <= ll^2 has a computed
 * per-axis |dx| <= ll (1 + 2^-23).  Without an image shift the computed
 * difference is within 2^-24 (relative) of the true one, so the true
 * separation stays below ll (1 + 2^-22): the relative term of the margin is
 * what keeps such a pair in neighbouring cells (a pair on a grid of side
 * exactly ll, whose difference rounds down onto ll, would otherwise sit two
 * cells apart).  With an image shift (x_i > x_j across the face) the computed
 * |dx| = L - fl(x_i - x_j) is at least L - x_i and exceeds x_j, since L - x_i
 * is a positive multiple of the ulp of x_i, so a pair two cells apart across
 * the face is never linked.  The absolute term L 2^-22 is further slack (by
 * itself it is at least three quarters of the relative one, as nc >= 3
 * below).  Every pair with computed D <= ll^2 is visited.
 */
static int fof3d_coarse(const float *x, const float *y, const float *z,
                        int64_t n, float L, float ll, int32_t *labels)
{
    double side_min = (double)ll * (1.0 + ldexp(1.0, -20)) + (double)L * ldexp(1.0, -22);
    int64_t nc = (int64_t)floor((double)L / side_min);
    if (nc < 3 || nc > 2000000) return oracle_fof3d_brute(x, y, z, n, L, ll, labels);
    float h = 0.5f * L, ll2 = ll * ll;
    double scale = (double)nc / (double)L;
    kv_t *s = (kv_t *)malloc(sizeof(kv_t) * (size_t)(n > 0 ? n : 1));
    int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!s || !parent) { free(s); free(parent); return -3; }
    for (int64_t i = 0; i < n; i++) {
        int64_t c[3];
        double u[3] = { (double)x[i] * scale, (double)y[i] * scale, (double)z[i] * scale };
        for (int a = 0; a < 3; a++) {
            c[a] = (int64_t)floor(u[a]);
            if (c[a] >= nc) c[a] = nc - 1;
            if (c[a] < 0) c[a] = 0;
        }
        s[i].key = (c[2] * nc + c[1]) * nc + c[0];
        s[i].idx = i;
        parent[i] = i;
    }
    qsort(s, (size_t)n, sizeof(kv_t), cmp_kv);
    int64_t start = 0;
    while (start < n) {
        int64_t key = s[start].key, end = start;
        while (end < n && s[end].key == key) end++;
        int64_t cx = key % nc, cy = (key / nc) % nc, cz = key / (nc * nc);
        for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++) {
            int64_t ox = (cx + dx + nc) % nc, oy = (cy + dy + nc) % nc, oz = (cz + dz + nc) % nc;
            int64_t nk = (oz * nc + oy) * nc + ox;
            if (nk < key) continue;          /* each cell pair once */
            int64_t b0 = lower_key(s, n, nk);
            for (int64_t p = start; p < end; p++)
                for (int64_t q = b0; q < n && s[q].key == nk; q++) {
                    if (nk == key && q <= p) continue;
                    if (pos_d2(x, y, z, s[p].idx, s[q].idx, L, h) <= ll2)
                        uf_union(parent, s[p].idx, s[q].idx);
                }
        }
        start = end;
    }
    for (int64_t i = 0; i < n; i++) labels[i] = (int32_t)uf_find(parent, i);
    free(s);
    free(parent);
    return 0;
}


/*
 * Periodic grid of small cells, side s = L / nc <= ll / sqrt(3 (1 + 1e-5)):
 * two particles of one cell are closer than the cell diagonal sqrt(3) s, so
 * their computed D <= ll^2 (the 1e-5 covers the rounding of the differences,
 * squares and sums, and of the fp64 cell assignment), and every particle of
 * a cell is linked to the cell's first one without a test.  A pair whose
 * computed D <= ll^2 has a true separation below ll (1 + 2^-22) + L 2^-24 on
 * every axis (the face argument of the coarse grid), so its cells are at most
 * r = floor((ll (1 + 2^-20) + L 2^-22) / s) + 1 apart per axis: each pair of
 * occupied cells within r is visited once, skipped when the two cells are
 * already one component, and otherwise linked at the first member pair with
 * D <= ll^2 (the two cells are each one component, so one link joins them).
 * Rows of cells (fixed y, z) are runs of the x-fastest keys, found through a
 * table of row starts.
 */
static int fof3d_fine(const float *x, const float *y, const float *z, int64_t n, float L,
                      float ll, int64_t nc, int64_t r, int32_t *labels)
{
    float h = 0.5f * L, ll2 = ll * ll;
    double scale = (double)nc / (double)L;
    kv_t *s = (kv_t *)malloc(sizeof(kv_t) * (size_t)(n > 0 ? n : 1));
    int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *rowstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc * nc + 1));
    if (!s || !parent || !rowstart) { free(s); free(parent); free(rowstart); return -3; }
    for (int64_t i = 0; i < n; i++) {
        int64_t c[3];
        double u[3] = { (double)x[i] * scale, (double)y[i] * scale, (double)z[i] * scale };
        for (int a = 0; a < 3; a++) {
            c[a] = (int64_t)floor(u[a]);
            if (c[a] >= nc) c[a] = nc - 1;
            if (c[a] < 0) c[a] = 0;
        }
        s[i].key = (c[2] * nc + c[1]) * nc + c[0];
        s[i].idx = i;
        parent[i] = i;
    }
    qsort(s, (size_t)n, sizeof(kv_t), cmp_kv);
    /* cells: runs of equal keys; every member joins the cell's first member */
    int64_t ncell = 0;
    for (int64_t p = 0; p < n; p++)
        if (p == 0 || s[p].key != s[p - 1].key) ncell++;
    int64_t *cfirst = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell + 1));
    int64_t *ckey = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell > 0 ? ncell : 1));
    if (!cfirst || !ckey) {
        free(s); free(parent); free(rowstart); free(cfirst); free(ckey);
        return -3;
    }
    int64_t k = 0;
    for (int64_t p = 0; p < n; p++) {
        if (p == 0 || s[p].key != s[p - 1].key) {
            cfirst[k] = p;
            ckey[k] = s[p].key;
            k++;
        } else {
            uf_union(parent, s[cfirst[k - 1]].idx, s[p].idx);
        }
    }
    cfirst[ncell] = n;
    /* rowstart[R] = first cell whose key is >= R nc */
    for (int64_t R = 0, c = 0; R <= nc * nc; R++) {
        while (c < ncell && ckey[c] < R * nc) c++;
        rowstart[R] = c;
    }
    for (int64_t a = 0; a < ncell; a++) {
        int64_t key = ckey[a];
        int64_t cx = key % nc, cy = (key / nc) % nc, cz = key / (nc * nc);
        int64_t pa = s[cfirst[a]].idx;
        for (int64_t dz = -r; dz <= r; dz++)
        for (int64_t dy = -r; dy <= r; dy++) {
            int64_t oy = (cy + dy + nc) % nc, oz = (cz + dz + nc) % nc;
            int64_t R = oz * nc + oy;
            for (int64_t b = rowstart[R]; b < rowstart[R + 1]; b++) {
                if (ckey[b] <= key) continue;               /* each cell pair once */
                int64_t ox = ckey[b] - R * nc;
                int64_t dxc = ox - cx;
                if (dxc > nc / 2) dxc -= nc;                /* x offset, nearest image */
                else if (dxc < -(nc / 2)) dxc += nc;
                if (dxc < -r || dxc > r) continue;
                int64_t pb = s[cfirst[b]].idx;
                if (uf_find(parent, pa) == uf_find(parent, pb)) continue;
                int found = 0;
                for (int64_t p = cfirst[a]; p < cfirst[a + 1] && !found; p++)
                    for (int64_t q = cfirst[b]; q < cfirst[b + 1]; q++)
                        if (pos_d2(x, y, z, s[p].idx, s[q].idx, L, h) <= ll2) {
                            found = 1;
                            break;
                        }
                if (found) uf_union(parent, pa, pb);
            }
        }
    }
    for (int64_t i = 0; i < n; i++) labels[i] = (int32_t)uf_find(parent, i);
    free(s); free(parent); free(rowstart); free(cfirst); free(ckey);
    return 0;
}

/*
 * 3D FoF of a periodic box.  mode 0: the small-cell grid with same-cell
 * linking where the grid allows it (at least 2r + 1 cells per axis and a
 * row table of at most 2^26 rows), else the coarse grid; 1: all pairs;
 * 2: the coarse grid (cells of side >= ll, every member pair of
 * neighbouring cells tested).
 */
int oracle_fof3d_mode(const float *x, const float *y, const float *z,
                      int64_t n, float L, float ll, int mode, int32_t *labels)
{
    if (n < 0 || !(L > 0.0f) || !(ll > 0.0f)) return -1;
    if (check_positions(x, y, z, n, L)) return -2;
    if (mode == 1) return oracle_fof3d_brute(x, y, z, n, L, ll, labels);
    if (mode == 0) {
        double smax = (double)ll / sqrt(3.0 * (1.0 + 1e-5));
        double cnt = ceil((double)L / smax);
        if (cnt <= 1048576.0) {
            int64_t nc = (int64_t)cnt;
            double side = (double)L / (double)nc;
            int64_t r = (int64_t)floor(((double)ll * (1.0 + ldexp(1.0, -20)) +
                                        (double)L * ldexp(1.0, -22)) / side) + 1;
            if (nc >= 2 * r + 1 && nc * nc <= ((int64_t)1 << 26))
                return fof3d_fine(x, y, z, n, L, ll, nc, r, labels);
        }
    }
    return fof3d_coarse(x, y, z, n, L, ll, labels);
}

int oracle_fof3d(const float *x, const float *y, const float *z,
                 int64_t n, float L, float ll, int32_t *labels)
{
    return oracle_fof3d_mode(x, y, z, n, L, ll, 0, labels);
}

/* ------------------------------------------------------------------ */
/* 3D FoF over a non-periodic sub-box with a ghost shell                */
/* ------------------------------------------------------------------ */

/*
 * The per-process FoF of the paper's decomposition (Parallelization
 * section): a process holds the particles of its sub-box [lo, hi) (owned,
 * indices [0, n_owned)) plus ghost copies of other processes' particles
 * within the shell [lo - gw, hi + gw) (indices [n_owned, n)).  No periodic
 * shift: D = fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz)) with dx = fl(xi - xj).
 * Labels are the smallest member index of each group.  Positions outside
 * their region (or non-finite) return -2.
 *
 * brute != 0 tests all pairs; otherwise a cell grid over the shell's
 * bounding cube with side >= ll (1 + 2^-20) + E 2^-22 (E the cube's side)
 * visits every pair in neighbouring cells (the margin argument of the
 * periodic grid, without the face).
 */
static int check_subbox(const float *x, const float *y, const float *z, int64_t n,
                        int64_t n_owned, const float *lo, const float *hi, float gw)
{
    const float *pc[3] = { x, y, z };
    for (int64_t i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) {
            float v = pc[a][i];
            if (i < n_owned) {
                if (!(v >= lo[a] && v < hi[a])) return -2;
            } else {
                double d = (double)v;
                if (!(d >= (double)lo[a] - (double)gw && d < (double)hi[a] + (double)gw)) return -2;
            }
        }
    return 0;
}

static float pos_d2_open(const float *x, const float *y, const float *z, int64_t i, int64_t j)
{
    float dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
    float sx = dx * dx, sy = dy * dy, sz = dz * dz;
    float t = sx + sy;
    return t + sz;
}

/*
 * The small-cell grid of the sub-box (no periodic images): cells of side
 * E / nc <= ll / sqrt(3 (1 + 1e-5)) over [o, o + E)^3, so that every pair in
 * one cell is within ll by any rounding and the cell's members are united
 * without tests; cell pairs up to r cells apart on every axis (the margin of
 * the coarse grid in cell units) are joined at their first linked member
 * pair, pairs already in one component skipped.  The same closure as
 * testing every pair.
 */
static int fof3d_fine_open(const float *x, const float *y, const float *z, int64_t n,
                           const double *o, double E, float ll, int64_t nc, int64_t r,
                           int32_t *labels)
{
    float ll2 = ll * ll;
    double scale = (double)nc / E;
    const float *pc[3] = { x, y, z };
    kv_t *s = (kv_t *)malloc(sizeof(kv_t) * (size_t)(n > 0 ? n : 1));
    int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *rowstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc * nc + 1));
    if (!s || !parent || !rowstart) { free(s); free(parent); free(rowstart); return -3; }
    for (int64_t i = 0; i < n; i++) {
        int64_t c[3];
        for (int a = 0; a < 3; a++) {
            c[a] = (int64_t)floor(((double)pc[a][i] - o[a]) * scale);
            if (c[a] >= nc) c[a] = nc - 1;
            if (c[a] < 0) c[a] = 0;
        }
        s[i].key = (c[2] * nc + c[1]) * nc + c[0];
        s[i].idx = i;
        parent[i] = i;
    }
    qsort(s, (size_t)n, sizeof(kv_t), cmp_kv);
    int64_t ncell = 0;
    for (int64_t p = 0; p < n; p++)
        if (p == 0 || s[p].key != s[p - 1].key) ncell++;
    int64_t *cfirst = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell + 1));
    int64_t *ckey = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell > 0 ? ncell : 1));
    if (!cfirst || !ckey) {
        free(s); free(parent); free(rowstart); free(cfirst); free(ckey);
        return -3;
    }
    int64_t k = 0;
    for (int64_t p = 0; p < n; p++) {
        if (p == 0 || s[p].key != s[p - 1].key) {
            cfirst[k] = p;
            ckey[k] = s[p].key;
            k++;
        } else {
            uf_union(parent, s[cfirst[k - 1]].idx, s[p].idx);
        }
    }
    cfirst[ncell] = n;
    for (int64_t R = 0, c = 0; R <= nc * nc; R++) {
        while (c < ncell && ckey[c] < R * nc) c++;
        rowstart[R] = c;
    }
    for (int64_t a = 0; a < ncell; a++) {
        int64_t key = ckey[a];
        int64_t cx = key % nc, cy = (key / nc) % nc, cz = key / (nc * nc);
        int64_t pa = s[cfirst[a]].idx;
        for (int64_t dz = -r; dz <= r; dz++)
        for (int64_t dy = -r; dy <= r; dy++) {
            int64_t oy = cy + dy, oz = cz + dz;
            if (oy < 0 || oz < 0 || oy >= nc || oz >= nc) continue;
            int64_t R = oz * nc + oy;
            for (int64_t b = rowstart[R]; b < rowstart[R + 1]; b++) {
                if (ckey[b] <= key) continue;               /* each cell pair once */
                int64_t dxc = (ckey[b] - R * nc) - cx;
                if (dxc < -r || dxc > r) continue;
                int64_t pb = s[cfirst[b]].idx;
                if (uf_find(parent, pa) == uf_find(parent, pb)) continue;
                int found = 0;
                for (int64_t p = cfirst[a]; p < cfirst[a + 1] && !found; p++)
                    for (int64_t q = cfirst[b]; q < cfirst[b + 1]; q++)
                        if (pos_d2_open(x, y, z, s[p].idx, s[q].idx) <= ll2) {
                            found = 1;
                            break;
                        }
                if (found) uf_union(parent, pa, pb);
            }
        }
    }
    for (int64_t i = 0; i < n; i++) labels[i] = (int32_t)uf_find(parent, i);
    free(s); free(parent); free(rowstart); free(cfirst); free(ckey);
    return 0;
}

/*
 * 3D FoF of a sub-box.  mode 0: the small-cell grid where it allows (at
 * least 2r + 1 cells per axis, a row table of at most 2^26 rows), else the
 * coarse grid; 1: all pairs; 2: the coarse grid (cells of side >= the
 * margin, every member pair of neighbouring cells tested).
 */
int oracle_fof3d_subbox_mode(const float *x, const float *y, const float *z, int64_t n,
                             int64_t n_owned, const float *lo, const float *hi, float gw,
                             float ll, int mode, int32_t *labels)
{
    if (n < 0 || n_owned < 0 || n_owned > n || !(ll > 0.0f) || !(gw >= 0.0f)) return -1;
    for (int a = 0; a < 3; a++)
        if (!(hi[a] > lo[a])) return -1;
    if (check_subbox(x, y, z, n, n_owned, lo, hi, gw)) return -2;
    float ll2 = ll * ll;
    double o[3], E = 0.0;
    for (int a = 0; a < 3; a++) {
        o[a] = (double)lo[a] - (double)gw;
        double e = ((double)hi[a] + (double)gw) - o[a];
        if (e > E) E = e;
    }
    double side_min = (double)ll * (1.0 + ldexp(1.0, -20)) + E * ldexp(1.0, -22);
    if (mode == 0) {
        double smax = (double)ll / sqrt(3.0 * (1.0 + 1e-5));
        double cnt = ceil(E / smax);
        if (cnt <= 1048576.0) {
            int64_t ncf = (int64_t)cnt;
            int64_t r = (int64_t)floor(side_min / (E / (double)ncf)) + 1;
            if (ncf >= 2 * r + 1 && ncf * ncf <= ((int64_t)1 << 26))
                return fof3d_fine_open(x, y, z, n, o, E, ll, ncf, r, labels);
        }
    }
    int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!parent) return -3;
    for (int64_t i = 0; i < n; i++) parent[i] = i;
    int64_t nc = (int64_t)floor(E / side_min);
    if (mode == 1 || nc < 3 || nc > 2000000) {
        for (int64_t i = 0; i < n; i++)
            for (int64_t j = i + 1; j < n; j++)
                if (pos_d2_open(x, y, z, i, j) <= ll2) uf_union(parent, i, j);
    } else {
        double scale = (double)nc / E;
        const float *pc[3] = { x, y, z };
        kv_t *s = (kv_t *)malloc(sizeof(kv_t) * (size_t)(n > 0 ? n : 1));
        if (!s) { free(parent); return -3; }
        for (int64_t i = 0; i < n; i++) {
            int64_t c[3];
            for (int a = 0; a < 3; a++) {
                c[a] = (int64_t)floor(((double)pc[a][i] - o[a]) * scale);
                if (c[a] >= nc) c[a] = nc - 1;
                if (c[a] < 0) c[a] = 0;
            }
            s[i].key = (c[2] * nc + c[1]) * nc + c[0];
            s[i].idx = i;
        }
        qsort(s, (size_t)n, sizeof(kv_t), cmp_kv);
        int64_t start = 0;
        while (start < n) {
            int64_t key = s[start].key, end = start;
            while (end < n && s[end].key == key) end++;
            int64_t cx = key % nc, cy = (key / nc) % nc, cz = key / (nc * nc);
            for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                int64_t ox = cx + dx, oy = cy + dy, oz = cz + dz;
                if (ox < 0 || oy < 0 || oz < 0 || ox >= nc || oy >= nc || oz >= nc) continue;
                int64_t nk = (oz * nc + oy) * nc + ox;
                if (nk < key) continue;          /* each cell pair once */
                int64_t b0 = lower_key(s, n, nk);
                for (int64_t p = start; p < end; p++)
                    for (int64_t q = b0; q < n && s[q].key == nk; q++) {
                        if (nk == key && q <= p) continue;
                        if (pos_d2_open(x, y, z, s[p].idx, s[q].idx) <= ll2)
                            uf_union(parent, s[p].idx, s[q].idx);
                    }
            }
            start = end;
        }
        free(s);
    }
    for (int64_t i = 0; i < n; i++) labels[i] = (int32_t)uf_find(parent, i);
    free(parent);
    return 0;
}

int oracle_fof3d_subbox(const float *x, const float *y, const float *z, int64_t n,
                        int64_t n_owned, const float *lo, const float *hi, float gw, float ll,
                        int brute, int32_t *labels)
{
    return oracle_fof3d_subbox_mode(x, y, z, n, n_owned, lo, hi, gw, ll, brute ? 1 : 0,
                                    labels);
}

/* ------------------------------------------------------------------ */
/* exact integer moments -> dispersions and metric factors             */
/* ------------------------------------------------------------------ */

/* Correctly rounded (nearest-even) conversion; gcc's own conversion. */
double oracle_i128_to_f64(int64_t hi, uint64_t lo)
{
    i128 v = ((i128)hi << 64) | (i128)lo;
    return (double)v;
}

typedef struct {
    float a, c;          /* 1/sigma_x^2, 1/sigma_v^2 (metric factors) */
    float sx2, sv2;      /* sigma_x^2, sigma_v^2 */
} norm_t;

/*
 * Positions quantised to Q = rint(x * 2^20) (fp64), taken relative to the
 * member with the smallest index and brought to the nearest periodic image
 * in integer arithmetic; velocities quantised to W = rint(v * 2^10).
 * Per axis S1 = sum(delta), S2 = sum(delta^2), exact in integers;
 * V = sum_axes (N*S2 - S1^2) = N^2 * (3D dispersion) in quantum units.
 */
static norm_t node_norm(const parts_t *p, const int64_t *mem, int64_t n, int64_t ref)
{
    const float *pc[3] = { p->x, p->y, p->z };
    const float *vc[3] = { p->vx, p->vy, p->vz };
    int64_t LQ = (int64_t)rint((double)p->L * 1048576.0);
    i128 Vx = 0, Vv = 0;
    for (int ax = 0; ax < 3; ax++) {
        int64_t qref = (int64_t)rint((double)pc[ax][ref] * 1048576.0);
        int64_t s1 = 0, t1 = 0;
        i128 s2 = 0, t2 = 0;
        for (int64_t m = 0; m < n; m++) {
            int64_t i = mem[m];
            int64_t d = (int64_t)rint((double)pc[ax][i] * 1048576.0) - qref;
            if (2 * d > LQ) d -= LQ;
            else if (2 * d <= -LQ) d += LQ;
            s1 += d;
            s2 += (i128)d * d;
            int64_t w = (int64_t)rint((double)vc[ax][i] * 1024.0);
            t1 += w;
            t2 += (i128)w * w;
        }
        Vx += (i128)n * s2 - (i128)s1 * s1;
        Vv += (i128)n * t2 - (i128)t1 * t1;
    }
    norm_t r;
    double nn = (double)n * (double)n;
    double vx = (double)Vx, vv = (double)Vv;
    r.a = (Vx == 0) ? 1.0f : (float)((nn / vx) * 1099511627776.0);   /* 2^40 */
    r.c = (Vv == 0) ? 1.0f : (float)((nn / vv) * 1048576.0);         /* 2^20 */
    r.sx2 = (float)((vx / nn) * 9.094947017729282e-13);              /* 2^-40 */
    r.sv2 = (float)((vv / nn) * 9.5367431640625e-07);                /* 2^-20 */
    return r;
}

/* ------------------------------------------------------------------ */
/* node-local 6D k-d tree (fp64 unwrapped coordinates)                 */
/* ------------------------------------------------------------------ */

/*
 * 6D k-d tree over one node's members: points are the positions unwrapped
 * around the reference member (fp64, exact differences of fp32 values) and
 * the raw velocities.  Each tree node covers a contiguous run of the slot
 * permutation (the root all n slots, children the two halves at the median
 * of the axis of largest metric-weighted extent) and stores the exact
 * bounding box of its points.  Leaves hold at most KD_LEAF slots.
 */
#define KD_LEAF 8

typedef struct {
    int64_t n;
    double *pt;          /* [n][6] */
    int64_t *idx;        /* slot permutation */
    double *box;         /* [nnode][12]: lo[6], hi[6] */
    int64_t nnode;
    float a, c;
    double slack;        /* absolute slack on position gaps */
} kd_t;

static void kd_free(kd_t *t)
{
    free(t->pt); free(t->idx); free(t->box);
    memset(t, 0, sizeof(*t));
}

/* place the m-th smallest coordinate (axis dim) of idx[b..e) at m */
static void kd_select(int64_t *idx, const double *pt, int dim, int64_t b, int64_t e, int64_t m)
{
    while (e - b > 1) {
        double v0 = pt[6 * idx[b] + dim], v1 = pt[6 * idx[b + (e - b) / 2] + dim],
               v2 = pt[6 * idx[e - 1] + dim];
        double piv = fmax(fmin(v0, v1), fmin(fmax(v0, v1), v2));   /* median of three */
        int64_t lt = b, i = b, gt = e;
        while (i < gt) {
            double v = pt[6 * idx[i] + dim];
            if (v < piv) { int64_t t = idx[lt]; idx[lt++] = idx[i]; idx[i++] = t; }
            else if (v > piv) { int64_t t = idx[--gt]; idx[gt] = idx[i]; idx[i] = t; }
            else i++;
        }
        if (m < lt) e = lt;
        else if (m >= gt) b = gt;
        else return;
    }
}

static void kd_build_node(kd_t *t, int64_t k, int64_t b, int64_t e)
{
    double *bx = t->box + 12 * k;
    for (int d = 0; d < 6; d++) { bx[d] = INFINITY; bx[6 + d] = -INFINITY; }
    for (int64_t i = b; i < e; i++) {
        const double *q = t->pt + 6 * t->idx[i];
        for (int d = 0; d < 6; d++) {
            if (q[d] < bx[d]) bx[d] = q[d];
            if (q[d] > bx[6 + d]) bx[6 + d] = q[d];
        }
    }
    if (e - b <= KD_LEAF) return;
    int dim = 0;
    double wmax = -1.0;
    for (int d = 0; d < 6; d++) {
        double w = (bx[6 + d] - bx[d]) * (d < 3 ? sqrt((double)t->a) : sqrt((double)t->c));
        if (w > wmax) { wmax = w; dim = d; }
    }
    int64_t m = b + (e - b) / 2;
    kd_select(t->idx, t->pt, dim, b, e, m);
    kd_build_node(t, 2 * k + 1, b, m);
    kd_build_node(t, 2 * k + 2, m, e);
}

/* Returns 0, or 1 if the node spans too much of the box for unwrapped
   coordinates (then the caller uses all pairs), -3 on allocation failure. */
static int kd_build(kd_t *t, const parts_t *p, const int64_t *mem, int64_t n, int64_t ref,
                    float a, float c)
{
    const float *pc[6] = { p->x, p->y, p->z, p->vx, p->vy, p->vz };
    double L = p->L;
    memset(t, 0, sizeof(*t));
    t->n = n; t->a = a; t->c = c;
    t->slack = 8.0 * L * ldexp(1.0, -23);
    int depth = 0;
    while (((n + ((int64_t)1 << depth) - 1) >> depth) > KD_LEAF) depth++;
    t->nnode = ((int64_t)1 << (depth + 1)) - 1;
    t->pt = (double *)malloc(sizeof(double) * 6 * (size_t)n);
    t->idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    t->box = (double *)malloc(sizeof(double) * 12 * (size_t)t->nnode);
    if (!t->pt || !t->idx || !t->box) { kd_free(t); return -3; }
    for (int d = 0; d < 3; d++) {
        double lo = INFINITY, hi = -INFINITY;
        for (int64_t m = 0; m < n; m++) {
            double u = (double)pc[d][mem[m]] - (double)pc[d][ref];
            if (u >= 0.5 * L) u -= L; else if (u < -0.5 * L) u += L;
            t->pt[6 * m + d] = u;
            if (u < lo) lo = u;
            if (u > hi) hi = u;
        }
        if (hi - lo > 0.25 * L) { kd_free(t); return 1; }
    }
    for (int d = 3; d < 6; d++)
        for (int64_t m = 0; m < n; m++) t->pt[6 * m + d] = (double)pc[d][mem[m]];
    for (int64_t m = 0; m < n; m++) t->idx[m] = m;
    kd_build_node(t, 0, 0, n);
    return 0;
}

/*
 * Lower bound on the computed d^2 between point q and any member inside tree
 * node k.  With the node extent below L/4 the unwrapped difference of two
 * members is their minimum-image difference, so each axis gap bounds |dx|
 * from below; position gaps lose an absolute slack (8 fp32 ulps of L) for
 * the rounding of the coordinate differences and image shift, and the sum
 * loses 1e-3 relative plus 1e-37 absolute for the rounding of squares, sums
 * and products (including subnormal results).
 */
static double kd_lb(const kd_t *t, int64_t k, const double *q)
{
    const double *bx = t->box + 12 * k;
    double sp = 0.0, sv = 0.0;
    for (int d = 0; d < 6; d++) {
        double g = fmax(fmax(bx[d] - q[d], q[d] - bx[6 + d]), 0.0);
        if (d < 3) { g = fmax(g - t->slack, 0.0); sp += g * g; }
        else sv += g * g;
    }
    return ((double)t->a * sp + (double)t->c * sv) * (1.0 - 1e-3) - 1e-37;
}

typedef struct {
    const kd_t *t;
    const parts_t *p;
    const int64_t *mem;
    int64_t self;
    const double *q;
    float best;          /* nearest-neighbour search */
    float l2;            /* linking */
    int64_t *parent;
} kd_query;

static void kd_nn(kd_query *s, int64_t k, int64_t b, int64_t e)
{
    if (kd_lb(s->t, k, s->q) >= (double)s->best) return;
    if (e - b <= KD_LEAF) {
        for (int64_t i = b; i < e; i++) {
            int64_t j = s->t->idx[i];
            if (j == s->self) continue;
            float d = phase_d2(s->p, s->mem[s->self], s->mem[j], s->t->a, s->t->c);
            if (d < s->best) s->best = d;
        }
        return;
    }
    int64_t m = b + (e - b) / 2;
    if (kd_lb(s->t, 2 * k + 1, s->q) <= kd_lb(s->t, 2 * k + 2, s->q)) {
        kd_nn(s, 2 * k + 1, b, m);
        kd_nn(s, 2 * k + 2, m, e);
    } else {
        kd_nn(s, 2 * k + 2, m, e);
        kd_nn(s, 2 * k + 1, b, m);
    }
}

/* unions the query with every later slot within l^2 */
static void kd_link(kd_query *s, int64_t k, int64_t b, int64_t e)
{
    if (kd_lb(s->t, k, s->q) > (double)s->l2) return;
    if (e - b <= KD_LEAF) {
        for (int64_t i = b; i < e; i++) {
            int64_t j = s->t->idx[i];
            if (j <= s->self) continue;
            if (phase_d2(s->p, s->mem[s->self], s->mem[j], s->t->a, s->t->c) <= s->l2)
                uf_union(s->parent, s->self, j);
        }
        return;
    }
    int64_t m = b + (e - b) / 2;
    kd_link(s, 2 * k + 1, b, m);
    kd_link(s, 2 * k + 2, m, e);
}

static int cmp_f32(const void *pa, const void *pb)
{
    float a = *(const float *)pa, b = *(const float *)pb;
    return (a > b) - (a < b);
}

/* k = ceil(f n) in exact integer arithmetic (f in parts per million), clamped. */
int64_t oracle_select_rank(int64_t n, double f)
{
    int64_t ppm = llround(f * 1e6);
    int64_t k = (n * ppm + 999999) / 1000000;
    if (k < 1) k = 1;
    if (k > n) k = n;
    return k;
}

/* ------------------------------------------------------------------ */
/* hierarchical 6D phase-space FoF                                     */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t *mem;        /* member indices, ascending */
    int64_t n;
    int32_t level;
    int64_t parent;      /* creation index of the parent, -1 for level 0 */
    float l2, a, c, sx2, sv2;
    int32_t wide;        /* the node's 3D group percolates (see group_wide) */
} node_t;

/*
 * Percolation flag of a 3D group: on some axis the members' integer
 * displacements from the reference member, brought to the nearest periodic
 * image exactly as for the dispersions, span at least half the box
 * (2 * (max - min) >= L_Q).  The nearest-image frame of such a group
 * is not unique, so its dispersions, and through them every node of its
 * hierarchy, are not invariant under translation; the children inherit it.
 */
static int32_t group_wide(const parts_t *p, const int64_t *mem, int64_t n, int64_t ref)
{
    const float *pc[3] = { p->x, p->y, p->z };
    int64_t LQ = (int64_t)rint((double)p->L * 1048576.0);
    for (int ax = 0; ax < 3; ax++) {
        int64_t qref = (int64_t)rint((double)pc[ax][ref] * 1048576.0);
        int64_t lo = 0, hi = 0;
        for (int64_t m = 0; m < n; m++) {
            int64_t d = (int64_t)rint((double)pc[ax][mem[m]] * 1048576.0) - qref;
            if (2 * d > LQ) d -= LQ;
            else if (2 * d <= -LQ) d += LQ;
            if (d < lo) lo = d;
            if (d > hi) hi = d;
        }
        if (2 * (hi - lo) >= LQ) return 1;
    }
    return 0;
}

typedef struct {
    node_t *v;
    int64_t n, cap;
} nodevec;

static int nv_push(nodevec *nv, node_t nd)
{
    if (nv->n == nv->cap) {
        int64_t nc = nv->cap ? 2 * nv->cap : 1024;
        node_t *t = (node_t *)realloc(nv->v, sizeof(node_t) * (size_t)nc);
        if (!t) return -3;
        nv->v = t; nv->cap = nc;
    }
    nv->v[nv->n++] = nd;
    return 0;
}

/*
 * Split one node: fills its l2/a/c/sigma fields and appends its children
 * (with member lists in ascending index order) to the node vector.
 * brute_max: nodes with at most this many members use all-pairs loops.
 */
static int split_node(nodevec *nv, int64_t id, const parts_t *p, int32_t min_sub,
                      double f, int64_t brute_max)
{
    node_t nd = nv->v[id];
    int64_t n = nd.n;
    const int64_t *mem = nd.mem;
    norm_t nm = node_norm(p, mem, n, mem[0]);       /* mem[0] is the smallest index */
    float a = nm.a, c = nm.c;

    float *d2 = (float *)malloc(sizeof(float) * (size_t)n);
    int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!d2 || !parent) { free(d2); free(parent); return -3; }

    kd_t t;
    int brute = (n <= brute_max);
    if (!brute) {
        brute = kd_build(&t, p, mem, n, mem[0], a, c);
        if (brute < 0) { free(d2); free(parent); return -3; }
    }

    /* nearest-neighbour distance of every member */
    if (brute) {
        for (int64_t i = 0; i < n; i++) {
            float best = INFINITY;
            for (int64_t j = 0; j < n; j++) {
                if (j == i) continue;
                float d = phase_d2(p, mem[i], mem[j], a, c);
                if (d < best) best = d;
            }
            d2[i] = best;
        }
    } else {
        for (int64_t i = 0; i < n; i++) {
            kd_query q = { &t, p, mem, i, t.pt + 6 * i, INFINITY, 0.0f, NULL };
            kd_nn(&q, 0, 0, n);
            d2[i] = q.best;
        }
    }

    /* the linking length: k-th smallest nearest-neighbour distance */
    int64_t k = oracle_select_rank(n, f);
    float *sorted = (float *)malloc(sizeof(float) * (size_t)n);
    memcpy(sorted, d2, sizeof(float) * (size_t)n);
    qsort(sorted, (size_t)n, sizeof(float), cmp_f32);
    float l2 = sorted[k - 1];
    free(sorted);

    /* link all pairs within l2 */
    for (int64_t i = 0; i < n; i++) parent[i] = i;
    if (brute) {
        for (int64_t i = 0; i < n; i++)
            for (int64_t j = i + 1; j < n; j++)
                if (phase_d2(p, mem[i], mem[j], a, c) <= l2) uf_union(parent, i, j);
    } else {
        for (int64_t i = 0; i < n; i++) {
            if (!(d2[i] <= l2)) continue;            /* no neighbour within l: cannot link */
            kd_query q = { &t, p, mem, i, t.pt + 6 * i, INFINITY, l2, parent };
            kd_link(&q, 0, 0, n);
        }
        kd_free(&t);
    }

    nv->v[id].l2 = l2; nv->v[id].a = a; nv->v[id].c = c;
    nv->v[id].sx2 = nm.sx2; nv->v[id].sv2 = nm.sv2;

    /* components; member slots are in ascending index order, so the root
       (smallest slot) is also the smallest particle index */
    int64_t *count = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) count[uf_find(parent, i)]++;
    int rc = 0;
    for (int64_t r = 0; r < n && rc == 0; r++) {
        if (parent[r] != r) continue;
        if (count[r] < min_sub || count[r] == n) continue;
        node_t ch;
        memset(&ch, 0, sizeof(ch));
        ch.n = count[r];
        ch.level = nd.level + 1;
        ch.parent = id;
        ch.wide = nd.wide;
        ch.mem = (int64_t *)malloc(sizeof(int64_t) * (size_t)ch.n);
        int64_t w = 0;
        for (int64_t i = r; i < n; i++)
            if (uf_find(parent, i) == r) ch.mem[w++] = mem[i];
        rc = nv_push(nv, ch);
    }
    free(count); free(d2); free(parent);
    return rc;
}

typedef struct { int64_t key; int64_t id; } nkey_t;

static int cmp_nkey(const void *pa, const void *pb)
{
    const nkey_t *a = (const nkey_t *)pa, *b = (const nkey_t *)pb;
    return (a->key > b->key) - (a->key < b->key);
}

/*
 * Full hierarchy.  Outputs (caller-allocated, capacity cap), canonical order
 * sorted by (level, smallest member index):
 *   level, min_index, parent (canonical index, -1 at level 0), size,
 *   l2, a, c, sx2, sv2, wide per node; deepest[n] = canonical index of the
 *   deepest node containing each particle, or -1.
 * Returns 0, -1 bad argument, -2 range, -3 memory, -4 capacity (n_nodes is
 * still written so the caller can retry).
 */
int oracle_phase_fof(const float *x, const float *y, const float *z,
                     const float *vx, const float *vy, const float *vz,
                     int64_t n, float L, const int32_t *fof_labels,
                     int32_t min_group, int32_t min_sub, double f, int64_t brute_max,
                     int64_t cap, int32_t *level, int32_t *min_index, int32_t *parent,
                     int32_t *size, float *l2, float *fa, float *fc, float *sx2, float *sv2,
                     int32_t *wide, int32_t *deepest, int64_t *n_nodes)
{
    if (n < 0 || !(L > 0.0f) || min_group < 2 || min_sub < 2 || !(f > 0.0 && f <= 1.0))
        return -1;
    if (check_positions(x, y, z, n, L)) return -2;
    for (int64_t i = 0; i < n; i++) {
        if (fof_labels[i] < 0 || fof_labels[i] >= n) return -1;
        if (!(fabsf(vx[i]) < 1048576.0f && fabsf(vy[i]) < 1048576.0f && fabsf(vz[i]) < 1048576.0f))
            return -2;
    }
    parts_t p = { x, y, z, vx, vy, vz, L, 0.5f * L };

    /* level-0 nodes: 3D groups with at least min_group members */
    int64_t *cnt = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) cnt[fof_labels[i]]++;
    nodevec nv = { 0, 0, 0 };
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++) slot[i] = -1;
    int rc = 0;
    for (int64_t r = 0; r < n && rc == 0; r++) {
        if (cnt[r] >= min_group) {
            node_t nd;
            memset(&nd, 0, sizeof(nd));
            nd.n = 0; nd.level = 0; nd.parent = -1;
            nd.mem = (int64_t *)malloc(sizeof(int64_t) * (size_t)cnt[r]);
            slot[r] = nv.n;
            rc = nv_push(&nv, nd);
        }
    }
    for (int64_t i = 0; i < n && rc == 0; i++) {
        int64_t s = slot[fof_labels[i]];
        if (s >= 0) nv.v[s].mem[nv.v[s].n++] = i;
    }
    free(cnt); free(slot);

    for (int64_t id = 0; id < nv.n && rc == 0; id++)
        nv.v[id].wide = group_wide(&p, nv.v[id].mem, nv.v[id].n, nv.v[id].mem[0]);
    for (int64_t id = 0; id < nv.n && rc == 0; id++)
        rc = split_node(&nv, id, &p, min_sub, f, brute_max);

    *n_nodes = nv.n;
    if (rc == 0 && nv.n > cap) rc = -4;
    if (rc == 0) {
        nkey_t *ord = (nkey_t *)malloc(sizeof(nkey_t) * (size_t)(nv.n > 0 ? nv.n : 1));
        int64_t *canon = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nv.n > 0 ? nv.n : 1));
        for (int64_t i = 0; i < nv.n; i++) {
            ord[i].key = ((int64_t)nv.v[i].level << 32) | nv.v[i].mem[0];
            ord[i].id = i;
        }
        qsort(ord, (size_t)nv.n, sizeof(nkey_t), cmp_nkey);
        for (int64_t r = 0; r < nv.n; r++) canon[ord[r].id] = r;
        for (int64_t i = 0; i < n; i++) deepest[i] = -1;
        for (int64_t r = 0; r < nv.n; r++) {
            node_t *nd = &nv.v[ord[r].id];
            level[r] = nd->level;
            min_index[r] = (int32_t)nd->mem[0];
            parent[r] = nd->parent < 0 ? -1 : (int32_t)canon[nd->parent];
            size[r] = (int32_t)nd->n;
            l2[r] = nd->l2; fa[r] = nd->a; fc[r] = nd->c;
            sx2[r] = nd->sx2; sv2[r] = nd->sv2;
            wide[r] = nd->wide;
            for (int64_t m = 0; m < nd->n; m++) deepest[nd->mem[m]] = (int32_t)r;
        }
        free(ord); free(canon);
    }
    for (int64_t i = 0; i < nv.n; i++) free(nv.v[i].mem);
    free(nv.v);
    return rc;
}

/* Nearest-neighbour distances of one explicit member set (for pins). */
int oracle_node_nn(const float *x, const float *y, const float *z,
                   const float *vx, const float *vy, const float *vz, float L,
                   const int64_t *mem, int64_t n, float a, float c, float *d2)
{
    parts_t p = { x, y, z, vx, vy, vz, L, 0.5f * L };
    for (int64_t i = 0; i < n; i++) {
        float best = INFINITY;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            float d = phase_d2(&p, mem[i], mem[j], a, c);
            if (d < best) best = d;
        }
        d2[i] = best;
    }
    return 0;
}

/* Metric factors of one explicit member set (mem ascending). */
int oracle_node_norm(const float *x, const float *y, const float *z,
                     const float *vx, const float *vy, const float *vz, float L,
                     const int64_t *mem, int64_t n, float *out4)
{
    parts_t p = { x, y, z, vx, vy, vz, L, 0.5f * L };
    norm_t r = node_norm(&p, mem, n, mem[0]);
    out4[0] = r.a; out4[1] = r.c; out4[2] = r.sx2; out4[3] = r.sv2;
    return 0;
}

/* ------------------------------------------------------------------ */
/* per-node halo properties                                            */
/* ------------------------------------------------------------------ */

/*
 * Properties of every node of a hierarchy (the halo properties, among them
 * the inertia tensor, that the paper's Summary lists among the new
 * functions).  A node's members are the particles whose deepest node is the
 * node or one of its descendants.  Positions are quantised to 2^-20 and
 * taken relative to the node's smallest-index member in the nearest periodic
 * image (as for the dispersions); velocities are quantised to 2^-10.  Per
 * node, in exact integers:
 *   S1_a = sum dQ_a, T1_a = sum W_a, S2_ab = sum dQ_a dQ_b,
 *   A_x = sum (dQ_y W_z - dQ_z W_y) (and cyclic),
 * then with nn = fl64(N) * fl64(N):
 *   centre_a   = ((double)Qref_a + (double)S1_a / (double)N) * 2^-20, moved
 *                into [0, L) by one shift of L in fp64, rounded to fp32 (a
 *                result equal to L is stored as 0);
 *   velocity_a = fl32(((double)T1_a / (double)N) * 2^-10);
 *   M_ab       = fl32((f64(N S2_ab - S1_a S1_b) / nn) * 2^-40), the second
 *                moment (shape, or inertia) tensor about the centre;
 *   j_a        = fl32((f64(N A_a - (S1_b T1_c - S1_c T1_b)) / nn) * 2^-30),
 *                (a, b, c) cyclic: the mean of (x - centre) x (v - velocity),
 *                the specific angular momentum about the centre.
 * f64() is the correctly rounded int128 -> fp64 conversion.
 * Output: props[q * n_nodes + k] for q in
 *   0..2 centre, 3..5 velocity, 6..11 Mxx Myy Mzz Mxy Mxz Myz, 12..14 j.
 * Returns 0, -1 (bad argument or inconsistent hierarchy), -3 (memory).
 */
int oracle_halo_props(const float *x, const float *y, const float *z,
                      const float *vx, const float *vy, const float *vz,
                      int64_t n, float L, int64_t n_nodes, const int32_t *parent,
                      const int32_t *min_index, const int32_t *deepest, float *props)
{
    if (n < 0 || n_nodes < 0 || !(L > 0.0f)) return -1;
    const float *pc[3] = { x, y, z };
    const float *vc[3] = { vx, vy, vz };
    int64_t LQ = (int64_t)rint((double)L * 1048576.0);
    /* members of each node: walk from each particle's deepest node to the root */
    int64_t *cnt = (int64_t *)calloc((size_t)(n_nodes + 1), sizeof(int64_t));
    if (!cnt) return -3;
    for (int64_t k = 0; k < n_nodes; k++)
        if (parent[k] >= n_nodes || parent[k] < -1 || min_index[k] < 0 || min_index[k] >= n) {
            free(cnt);
            return -1;
        }
    for (int64_t i = 0; i < n; i++) {
        if (deepest[i] < -1 || deepest[i] >= n_nodes) { free(cnt); return -1; }
        int64_t depth = 0;
        for (int64_t k = deepest[i]; k >= 0; k = parent[k]) {
            cnt[k]++;
            if (++depth > n_nodes) { free(cnt); return -1; }   /* a cycle */
        }
    }
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_nodes + 1));
    int64_t *fill = (int64_t *)calloc((size_t)(n_nodes + 1), sizeof(int64_t));
    if (!start || !fill) { free(cnt); free(start); free(fill); return -3; }
    start[0] = 0;
    for (int64_t k = 0; k < n_nodes; k++) start[k + 1] = start[k] + cnt[k];
    int64_t *mem = (int64_t *)malloc(sizeof(int64_t) * (size_t)(start[n_nodes] > 0 ? start[n_nodes] : 1));
    if (!mem) { free(cnt); free(start); free(fill); return -3; }
    for (int64_t i = 0; i < n; i++)
        for (int64_t k = deepest[i]; k >= 0; k = parent[k]) mem[start[k] + fill[k]++] = i;

    for (int64_t k = 0; k < n_nodes; k++) {
        int64_t N = cnt[k];
        const int64_t *m = mem + start[k];
        int64_t ref = min_index[k];
        int64_t s1[3] = { 0, 0, 0 }, t1[3] = { 0, 0, 0 }, qref[3];
        i128 s2[3][3], an[3] = { 0, 0, 0 };
        for (int a = 0; a < 3; a++) {
            qref[a] = (int64_t)rint((double)pc[a][ref] * 1048576.0);
            for (int b = 0; b < 3; b++) s2[a][b] = 0;
        }
        for (int64_t t = 0; t < N; t++) {
            int64_t i = m[t], d[3], w[3];
            for (int a = 0; a < 3; a++) {
                d[a] = (int64_t)rint((double)pc[a][i] * 1048576.0) - qref[a];
                if (2 * d[a] > LQ) d[a] -= LQ;
                else if (2 * d[a] <= -LQ) d[a] += LQ;
                w[a] = (int64_t)rint((double)vc[a][i] * 1024.0);
                s1[a] += d[a];
                t1[a] += w[a];
            }
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) s2[a][b] += (i128)d[a] * d[b];
            for (int a = 0; a < 3; a++) {
                int b = (a + 1) % 3, c = (a + 2) % 3;
                an[a] += (i128)d[b] * w[c] - (i128)d[c] * w[b];
            }
        }
        float out[15];
        if (N == 0) {
            for (int q = 0; q < 15; q++) out[q] = 0.0f;
        } else {
            double nn = (double)N * (double)N;
            for (int a = 0; a < 3; a++) {
                double u = ((double)qref[a] + (double)s1[a] / (double)N) * 9.5367431640625e-07;
                if (u < 0.0) u += (double)L;
                else if (u >= (double)L) u -= (double)L;
                float c = (float)u;
                out[a] = (c >= L) ? 0.0f : c;
                out[3 + a] = (float)(((double)t1[a] / (double)N) * 9.765625e-4);
            }
            static const int pa[6] = { 0, 1, 2, 0, 0, 1 }, pb[6] = { 0, 1, 2, 1, 2, 2 };
            for (int q = 0; q < 6; q++) {
                int a = pa[q], b = pb[q];
                i128 cm = (i128)N * s2[a][b] - (i128)s1[a] * s1[b];
                out[6 + q] = (float)(((double)cm / nn) * 9.094947017729282e-13);   /* 2^-40 */
            }
            for (int a = 0; a < 3; a++) {
                int b = (a + 1) % 3, c = (a + 2) % 3;
                i128 jn = (i128)N * an[a] - ((i128)s1[b] * t1[c] - (i128)s1[c] * t1[b]);
                out[12 + a] = (float)(((double)jn / nn) * 9.313225746154785e-10);  /* 2^-30 */
            }
        }
        for (int q = 0; q < 15; q++) props[q * n_nodes + k] = out[q];
    }
    free(cnt); free(start); free(fill); free(mem);
    return 0;
}

/* ------------------------------------------------------------------ */
/* seed-halo assignment                                                */
/* ------------------------------------------------------------------ */

/*
 * Completes the hierarchy into a particle-to-halo assignment (the rest of
 * the subhalo finding the paper's Parallelization section attributes to the
 * 6D phase-space step; the reading is stated in full in the design notes).
 * Seeds are the leaves of the hierarchy (nodes without children).  A
 * particle whose deepest node is a seed belongs to it; a particle whose
 * deepest node d has children goes to the seed s, among the seeds in d's
 * subtree, with the smallest
 *   d^2 = fl(fl(a_s * Dx) + fl(c_s * Dv)),
 * Dx the fp32 sum ((dx^2 + dy^2) + dz^2) of the nearest-image differences
 * x_p - centre_s (one periodic shift per axis), Dv the same sum over
 * v_p - velocity_s without a shift, a_s and c_s the seed's metric factors;
 * ties go to the smaller node index.  Particles outside every node get -1.
 * props holds the node properties (oracle_halo_props layout: centre in rows
 * 0..2, bulk velocity in rows 3..5).  Returns 0, -1 (inconsistent input) or
 * -3 (memory).
 */
int oracle_seed_assign(const float *x, const float *y, const float *z,
                       const float *vx, const float *vy, const float *vz, int64_t n, float L,
                       int64_t n_nodes, const int32_t *parent, const int32_t *deepest,
                       const float *fa, const float *fc, const float *props, int32_t *halo)
{
    if (n < 0 || n_nodes < 0 || !(L > 0.0f)) return -1;
    float h = 0.5f * L;
    int64_t *nkid = (int64_t *)calloc((size_t)(n_nodes + 1), sizeof(int64_t));
    if (!nkid) return -3;
    for (int64_t k = 0; k < n_nodes; k++) {
        if (parent[k] < -1 || parent[k] >= n_nodes) { free(nkid); return -1; }
        if (parent[k] >= 0) nkid[parent[k]]++;
    }
    /* the seeds of each node's subtree: every leaf is listed under itself and
       each of its ancestors */
    int64_t *cnt = (int64_t *)calloc((size_t)(n_nodes + 1), sizeof(int64_t));
    int64_t *start = (int64_t *)calloc((size_t)(n_nodes + 1), sizeof(int64_t));
    int64_t *fill = (int64_t *)calloc((size_t)(n_nodes + 1), sizeof(int64_t));
    if (!cnt || !start || !fill) { free(nkid); free(cnt); free(start); free(fill); return -3; }
    for (int64_t s = 0; s < n_nodes; s++) {
        if (nkid[s]) continue;
        int64_t depth = 0;
        for (int64_t k = s; k >= 0; k = parent[k]) {
            cnt[k]++;
            if (++depth > n_nodes) { free(nkid); free(cnt); free(start); free(fill); return -1; }
        }
    }
    for (int64_t k = 0; k < n_nodes; k++) start[k + 1] = start[k] + cnt[k];
    int64_t *seeds = (int64_t *)malloc(sizeof(int64_t) * (size_t)(start[n_nodes] > 0 ? start[n_nodes] : 1));
    if (!seeds) { free(nkid); free(cnt); free(start); free(fill); return -3; }
    for (int64_t s = 0; s < n_nodes; s++) {
        if (nkid[s]) continue;
        for (int64_t k = s; k >= 0; k = parent[k]) seeds[start[k] + fill[k]++] = s;
    }
    for (int64_t i = 0; i < n; i++) {
        int64_t d = deepest[i];
        if (d < -1 || d >= n_nodes) { halo[i] = -1; continue; }
        if (d < 0) { halo[i] = -1; continue; }
        if (!nkid[d]) { halo[i] = (int32_t)d; continue; }
        float best = INFINITY;
        int64_t bs = -1;
        for (int64_t t = start[d]; t < start[d + 1]; t++) {
            int64_t s = seeds[t];
            float dx = min_image(x[i] - props[0 * n_nodes + s], L, h);
            float dy = min_image(y[i] - props[1 * n_nodes + s], L, h);
            float dz = min_image(z[i] - props[2 * n_nodes + s], L, h);
            float sx = dx * dx, sy = dy * dy, sz = dz * dz;
            float t1 = sx + sy;
            float Dx = t1 + sz;
            float du = vx[i] - props[3 * n_nodes + s];
            float dv = vy[i] - props[4 * n_nodes + s];
            float dw = vz[i] - props[5 * n_nodes + s];
            float su = du * du, sv = dv * dv, sw = dw * dw;
            float t2 = su + sv;
            float Dv = t2 + sw;
            float u = fa[s] * Dx, w = fc[s] * Dv;
            float d2 = u + w;
            if (d2 < best || (d2 == best && s < bs)) { best = d2; bs = s; }
        }
        halo[i] = (int32_t)bs;
    }
    free(nkid); free(cnt); free(start); free(fill); free(seeds);
    return 0;
}
