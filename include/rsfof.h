/*
 * rsfof.h -- C ABI of the MI355X friends-of-friends halo-finding core.
 *
 * The library implements the two data-parallel steps that the MPI-Rockstar
 * paper (arXiv:2412.18629, Parallelization section) describes for each
 * process's sub-box: a 3D friends-of-friends pass that finds overdense
 * regions, then subhalo finding inside every FoF halo using 6D phase-space
 * information (Rockstar's hierarchical phase-space FoF, the method the paper
 * cites in its Summary).  All compute runs in HIP kernels for gfx950.
 *
 * Conventions shared by every entry point:
 *   - Pointers are DEVICE pointers unless marked (host).
 *   - Inputs are caller-owned and only read.  Positions are fp32 SoA arrays
 *     x[n], y[n], z[n] in [0, box); velocities are fp32 SoA vx[n], vy[n],
 *     vz[n] in km/s with |v| < 2^20.
 *   - Argument errors are reported before any device work.  On any error
 *     the return value is negative, outputs are left untouched, and nothing
 *     leaks.  Out-of-range or non-finite coordinates are detected on the
 *     device before any output is written and reported as RS_ERANGE.
 *   - `stream` is a hipStream_t (NULL = the default stream).  The library
 *     keeps one grow-only workspace per device.  Calls on one device from
 *     several host threads are serialised by a per-device lock (each holds it
 *     until it returns); the stream-ordered rs_mlp_train_step and
 *     rs_sort_pairs_u64_i32 may still have work in flight after returning,
 *     so they must not overlap other calls on other streams of that device.
 *
 * Pair arithmetic (fixed, identical in every kernel):
 *   dx = fl(xi - xj) followed by one periodic shift (dx > box/2: dx - box;
 *   dx < -box/2: dx + box); D = fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz)),
 *   no fused multiply-add, round to nearest even, denormals kept.
 */
#ifndef RSFOF_H
#define RSFOF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RS_OK = 0,
    RS_EINVAL = -1,     /* bad argument (NULL pointer, size, parameter range) */
    RS_ERANGE = -2,     /* a coordinate outside [0, box), non-finite, or |v| >= 2^20 */
    RS_ENOMEM = -3,     /* device allocation failed */
    RS_EDEVICE = -4,    /* no usable HIP device, or a HIP runtime error */
    RS_EINTERNAL = -5,  /* internal capacity or consistency failure */
    RS_ENOTIMPL = -6    /* requested mode not available */
} rs_status;

/* Execution forms of rs_phase_fof_batch.  All forms return identical results. */
enum {
    RS_PLAIN = 0,    /* one level-0 group per launch sequence, host-driven */
    RS_BATCHED = 1,  /* all groups and levels through size-bucketed kernels */
    RS_LEARNED = 2,  /* batched, linking length proposed by the MLP and verified
                        by exact counting in a bracket (implies RS_BATCHED) */
    RS_FEATURES = 0x100  /* OR-able: also return the per-node proposer features */
};

/* Proposer features per node (float): [0] ln N; [1..3] per-axis share of the
 * position dispersion; [4..6] per-axis share of the velocity dispersion;
 * [7..14] fractions of members with |x - mean| / sigma_x in the bins with
 * edges {0.25, 0.5, 0.75, 1, 1.5, 2, 3}; [15..22] the same for
 * |v - mean| / sigma_v; [23] recursion level. */
#define RS_NFEAT 24
/* MLP parameters: W1[64][24], b1[64], W2[64][64], b2[64], W3[64], b3 */
#define RS_MLP_NPARAM 5825
/* Size of the proposer blob rs_phase_fof_batch takes: "RSM1" + float32
 * mean[RS_NFEAT], std[RS_NFEAT], params[RS_MLP_NPARAM]. */
#define RS_MODEL_BYTES (4 + 4 * (2 * RS_NFEAT + RS_MLP_NPARAM))

/*
 * rs_fof3d -- 3D friends-of-friends over one periodic box (the per-process
 * FoF pass of the paper's Parallelization section).
 *
 * Groups are the connected components of the pair relation D(i,j) <= ll^2
 * with ll = link_len (an absolute length; a caller following the paper's
 * convention passes b times the mean interparticle spacing).
 *   x, y, z    [n] fp32 positions, 0 <= x < box.
 *   n          0 <= n < 2^31.
 *   box        periodic box side, > 0.
 *   link_len   0 < link_len < box / 2.
 *   labels     [n] int32 output, caller-allocated: the smallest particle
 *              index of each particle's group.
 *   n_groups   (host, optional) number of groups, including singletons.
 * Synchronous with respect to `stream` on return.
 */
int rs_fof3d(const float* x, const float* y, const float* z, int64_t n,
             float box, float link_len, int32_t* labels, int64_t* n_groups,
             void* stream);

/*
 * rs_fof3d_noalloc -- rs_fof3d for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, checks, results and synchronisation as rs_fof3d (it reads
 * counters back mid-pass, so like rs_fof3d it cannot be recorded into a
 * graph), but the pass's work space is a fixed 128 MiB device array
 * (RS_NOALLOC_SCRATCH_BYTES) that each GPU the library runs on holds from the
 * library's load until the process ends; the call allocates nothing.  A pass
 * needs about 110 bytes per particle (its sort, tables, union-find and the
 * grid's row table): about 1.1 million particles fit, and a call that needs
 * more returns RS_EINVAL before any device work.  Every call on one GPU
 * shares that GPU's array (whatever an earlier call left there is cleared or
 * overwritten before use).  Calls from several host threads are serialised
 * by the per-device lock, so they never overlap on the array.
 */
#define RS_NOALLOC_SCRATCH_BYTES (128u << 20)
int rs_fof3d_noalloc(const float* x, const float* y, const float* z, int64_t n, float box,
                     float link_len, int32_t* labels, int64_t* n_groups, void* stream);

/*
 * rs_fof3d_subbox -- 3D friends-of-friends over one process's non-periodic
 * sub-box with a ghost shell (the paper's decomposition, Parallelization
 * section: each process runs the 3D FoF over its own sub-box, and halos are
 * then joined across processes through the particles near the boundaries).
 *
 * Particles [0, n_owned) are the process's own and lie in [lo, hi) per
 * axis; particles [n_owned, n) are ghost copies of other processes'
 * particles (periodic images shifted into this frame, as the caller
 * decomposes the box) in the shell [lo - ghost_width, hi + ghost_width).
 * Groups are the connected components of D(i,j) <= link_len^2 over all n
 * particles, with the pair arithmetic of rs_fof3d WITHOUT the periodic
 * shift.  For the union across processes to find every link, ghost_width
 * must exceed link_len (by any margin above 2^-20 relative).
 *   lo, hi       (host) float[3], lo < hi.
 *   ghost_width  >= 0.
 *   link_len     > 0.
 *   labels       [n] int32 output: the smallest index (in this call's
 *                numbering) of each particle's group.
 *   ghost_links  [2 * (n - n_owned)] int32 output or NULL: pairs
 *                (ghost index, its label) for every ghost whose group holds
 *                an owned particle (label < n_owned), by ghost index; the
 *                cross-process union joins the ghost's own process's group
 *                with this one through them.
 *   n_links      (host) number of pairs; required with ghost_links.
 * Positions outside their region or not finite: RS_ERANGE.  Synchronous with
 * respect to `stream` on return.
 */
int rs_fof3d_subbox(const float* x, const float* y, const float* z, int64_t n, int64_t n_owned,
                    const float* lo, const float* hi, float ghost_width, float link_len,
                    int32_t* labels, int32_t* ghost_links, int64_t* n_links, void* stream);

/*
 * Node hierarchy returned by rs_phase_fof_batch.  The struct lives in host
 * memory; every array lives in ONE library-owned device allocation, released
 * only by rs_free.
 *
 * Nodes are in canonical order, sorted by (level, min_index).  A level-0
 * node is a 3D group with at least min_group members; a node's children are
 * the components (>= min_sub members, not the whole node) of its 6D split.
 */
typedef struct rs_tree {
    int64_t n_nodes;
    int64_t n_particles;
    int32_t* level;      /* [n_nodes] recursion depth, 0 for a 3D group */
    int32_t* min_index;  /* [n_nodes] smallest member particle index */
    int32_t* parent;     /* [n_nodes] index of the parent node, -1 at level 0 */
    int32_t* size;       /* [n_nodes] member count */
    float* l2;           /* [n_nodes] squared 6D linking length that split the node */
    float* a;            /* [n_nodes] position metric factor 1/sigma_x^2 */
    float* c;            /* [n_nodes] velocity metric factor 1/sigma_v^2 */
    float* sx2;          /* [n_nodes] position dispersion sigma_x^2, (Mpc/h)^2 */
    float* sv2;          /* [n_nodes] velocity dispersion sigma_v^2, (km/s)^2 */
    int32_t* deepest;    /* [n_particles] deepest node containing the particle, or -1 */
    int64_t n_accepted;  /* RS_LEARNED: nodes whose proposed bracket held */
    int64_t n_fallback;  /* RS_LEARNED: nodes whose bracket was rejected and which
                            were completed by the exact refinement */
    int64_t n_levels;    /* number of levels (max level + 1), 0 if no nodes */
    float* features;     /* [n_nodes * RS_NFEAT] with RS_FEATURES, else NULL */
    int32_t* wide;       /* [n_nodes] 1 when the node's 3D group percolates: on some
                            axis its members' integer displacements from the group's
                            smallest-index member (nearest periodic image, as for the
                            dispersions) span at least half the box, so the group's
                            nearest-image frame, and with it every node of its
                            hierarchy, is not translation invariant; else 0 */
} rs_tree;

/*
 * rs_phase_fof_batch -- hierarchical 6D phase-space FoF inside every 3D group
 * (paper, Parallelization section: subhalo finding for each FoF halo using
 * 6D phase-space information; method of the cited Rockstar paper).
 *
 * For each node: dispersions sigma_x^2, sigma_v^2 from exact integer moments
 * (positions quantised to 2^-20 relative to the node's smallest-index member
 * in the nearest periodic image, velocities to 2^-10); metric
 * d^2 = fl(fl(a*Dx) + fl(c*Dv)), a = 1/sigma_x^2, c = 1/sigma_v^2 (fp32);
 * l^2 = the k-th smallest nearest-neighbour d^2 of the members, k = ceil(f n);
 * members are linked when d^2 <= l^2; components of >= min_sub members other
 * than the whole node become children and are split in turn.
 *
 *   x..vz       [n] fp32 positions and velocities.
 *   fof_labels  [n] int32 group ids in [0, n) (rs_fof3d labels).
 *   min_group   >= 2, smallest 3D group that is split (paper configs: 10).
 *   min_sub     >= 2, smallest child kept (10).
 *   f           0 < f <= 1, linked fraction (0.7).
 *   flags       RS_PLAIN, RS_BATCHED or RS_LEARNED, optionally | RS_FEATURES.
 *   model       (host) proposer blob of RS_MODEL_BYTES bytes ("RSM1" + floats,
 *               see below) for RS_LEARNED, else NULL; only the tag is checked,
 *               so a shorter buffer is read past its end.  RS_LEARNED applies the proposal to
 *               nodes above the workgroup size (2048 members); smaller nodes
 *               are split exactly as in RS_BATCHED.
 *   out         (host) receives a new rs_tree* (release with rs_free).
 * Returns after synchronising `stream`.
 */
int rs_phase_fof_batch(const float* x, const float* y, const float* z,
                       const float* vx, const float* vy, const float* vz,
                       int64_t n, float box, const int32_t* fof_labels,
                       int32_t min_group, int32_t min_sub, double f,
                       uint32_t flags, const void* model, rs_tree** out,
                       void* stream);

/*
 * rs_halo_props -- per-node halo properties over a hierarchy returned by
 * rs_phase_fof_batch (the halo properties, inertia tensor among them, that
 * the paper's Summary lists among MPI-Rockstar's new functions).
 *
 * A node's members are the particles whose deepest node is the node or one
 * of its descendants.  Positions are quantised to 2^-20 and taken relative
 * to the node's smallest-index member (min_index) in the nearest periodic
 * image, velocities quantised to 2^-10; all sums are exact integers, so the
 * result does not depend on member order.  Per node (N members):
 *   centre   ((double)Q_ref + (double)sum(dQ) / N) * 2^-20 (fp64), moved into
 *            [0, box) by one shift of box, rounded to fp32 (box is stored as 0);
 *   velocity fl32(((double)sum(W) / N) * 2^-10), the bulk velocity;
 *   M_ab     fl32((f64(N sum(dQ_a dQ_b) - sum(dQ_a) sum(dQ_b)) / (N N)) * 2^-40),
 *            the second-moment (shape, inertia) tensor about the centre;
 *   j_a      fl32((f64(N sum(dQ_b W_c - dQ_c W_b) - (sum(dQ_b) sum(W_c) -
 *            sum(dQ_c) sum(W_b))) / (N N)) * 2^-30), (a, b, c) cyclic: the mean
 *            of (x - centre) x (v - velocity), the specific angular momentum.
 *
 *   x..vz       [n] fp32 positions (0 <= x < box) and velocities (|v| < 2^20).
 *   box         periodic box side, 0 < box < 2048 (quantised coordinates and
 *               their 128-bit moments stay exact below that).
 *   n_nodes, n_levels, level, parent, min_index, size, deepest: the hierarchy
 *               exactly as rs_tree holds it (canonical order; deepest [n]).
 *   props       [RS_NPROP * n_nodes] fp32 output, caller-allocated, row-major
 *               by property: props[q * n_nodes + k], q in RS_PROP_* order.
 * The hierarchy is checked on the device (levels sorted, each parent one
 * level up and earlier, child sizes within the parent, every node's own
 * particles exactly size minus its children's sizes): RS_EINVAL otherwise,
 * before any output is written.  Uses the library's workspace; returns after
 * synchronising `stream`.  RS_OK, RS_EINVAL, RS_ERANGE, RS_ENOMEM, RS_EDEVICE.
 */
enum {
    RS_PROP_CX = 0, RS_PROP_CY, RS_PROP_CZ,        /* centre */
    RS_PROP_VX, RS_PROP_VY, RS_PROP_VZ,            /* bulk velocity */
    RS_PROP_MXX, RS_PROP_MYY, RS_PROP_MZZ,         /* second-moment tensor */
    RS_PROP_MXY, RS_PROP_MXZ, RS_PROP_MYZ,
    RS_PROP_JX, RS_PROP_JY, RS_PROP_JZ,            /* specific angular momentum */
    RS_NPROP
};
int rs_halo_props(const float* x, const float* y, const float* z, const float* vx,
                  const float* vy, const float* vz, int64_t n, float box, int64_t n_nodes,
                  int64_t n_levels, const int32_t* level, const int32_t* parent,
                  const int32_t* min_index, const int32_t* size, const int32_t* deepest,
                  float* props, void* stream);

/*
 * rs_seed_assign -- assigns every particle of a hierarchy to a seed halo,
 * completing the subhalo finding of the 6D phase-space step (paper,
 * Parallelization section; the method is deferred there to the cited
 * Rockstar paper, so this follows a stated reading):
 *   seeds are the leaves of the hierarchy (nodes without children); a
 *   particle whose deepest node is a seed belongs to it; a particle whose
 *   deepest node d has children goes to the seed s below d with the smallest
 *   d^2 = fl(fl(a_s * Dx) + fl(c_s * Dv)), Dx the fp32 sum ((dx^2 + dy^2) +
 *   dz^2) of the nearest-image differences x - centre_s, Dv the same sum of
 *   v - velocity_s without a shift; ties go to the smaller node index.
 *   x..vz       [n] fp32 positions (0 <= x < box) and velocities.
 *   n_nodes ... deepest, a, c: the hierarchy exactly as rs_tree holds it.
 *   props       [RS_NPROP * n_nodes] as rs_halo_props returns it (centre and
 *               bulk velocity are read).
 *   halo        [n] int32 output: the seed's node index, -1 outside every node.
 * The hierarchy is checked as in rs_halo_props (RS_EINVAL before any output
 * is written); uses the library's workspace and returns after synchronising
 * `stream`.  RS_OK, RS_EINVAL, RS_ERANGE, RS_ENOMEM, RS_EDEVICE.
 */
int rs_seed_assign(const float* x, const float* y, const float* z, const float* vx,
                   const float* vy, const float* vz, int64_t n, float box, int64_t n_nodes,
                   int64_t n_levels, const int32_t* level, const int32_t* parent,
                   const int32_t* min_index, const int32_t* size, const int32_t* deepest,
                   const float* a, const float* c, const float* props, int32_t* halo,
                   void* stream);

/*
 * Linking-length proposer: a small network that predicts ln l of a node from
 * 24 summary features.  It never decides a result: RS_LEARNED verifies every
 * proposal exactly and completes rejected ones with the exact search.  All
 * pointers are device pointers.
 *
 * rs_mlp_forward:   y[n] = MLP(params, X[n][RS_NFEAT]) in fp32 (X standardised).
 * rs_mlp_grad:      grad[RS_MLP_NPARAM] and loss = mean((y - t)^2) over n samples.
 * rs_mlp_train_step: one Adam step (lr, beta 0.9/0.999, eps 1e-8; `step` >= 1
 *                   is the 1-based step count) on params with moments m, v;
 *                   writes the minibatch loss before the update to *loss.
 * rs_mlp_standardize: X <- (X - mean) / std per feature; with compute != 0
 *                   mean and std are first computed from X (std 1 if ~0).
 * rs_mlp_infer:     out[n] = MLP(model, features) with bf16 weights and
 *                   activations and fp32 accumulation; model = mean[24],
 *                   std[24], params[RS_MLP_NPARAM]; features unstandardised.
 * rs_phase_fof_batch's `model` (host) is that same float layout preceded by
 * the 4-byte tag "RSM1".  Each returns RS_OK or RS_EINVAL / RS_EDEVICE.
 */
int rs_mlp_forward(const float* params, const float* X, int64_t n, float* y, void* stream);
int rs_mlp_grad(const float* params, const float* X, const float* t, int64_t n, float* grad,
                float* loss, void* stream);
int rs_mlp_train_step(float* params, float* m, float* v, int64_t step, const float* X,
                      const float* t, int64_t n, float lr, float* loss, void* stream);
int rs_mlp_standardize(float* X, int64_t n, float* mean, float* stdv, int compute, void* stream);
int rs_mlp_infer(const float* model, int64_t n, const float* features, float* out, void* stream);

/*
 * Instrumentation (not part of the method).  While enabled, the library
 * records HIP events on the launching stream around its main kernels
 * ("fof3d_link", "phase_small", "phase_large_nn", "phase_large_link",
 * "phase_large_nn_fallback", "halo_props", "seed_assign") and
 * accumulates their elapsed time, launch count and processed work units
 * (particles or node members).  rs_profile_enable(0) clears the records.
 * rs_profile_enable(2) also counts the pair tests of the searches, reported
 * as units of "pairs_fof3d" (member pairs of octant pairs tested in the 3D
 * link), "pairs_nn" (query-member pairs evaluated by the large-node
 * nearest-neighbour searches, refinements included) and "pairs_link" (pairs
 * of a query and a later member evaluated by the large-node link), launches
 * counted, no time.  Counting runs slower kernel builds and synchronises
 * after each counted launch: for measurement runs, not timed ones.
 * rs_profile_get synchronises on the recorded events; unknown names report
 * zeros.  Returns RS_OK, or RS_EINVAL for NULL arguments.
 */
int rs_profile_enable(int on);
int rs_profile_get(const char* name, double* total_ms, int64_t* launches, double* units);

/*
 * Stable key/value sort, the primitive behind the cell-sorted layout of the
 * 3D pass and the per-node member orders of the 6D pass (the per-process
 * steps of the Parallelization section).  Sorts (keys_in[i], vals_in[i]) by
 * the low `bits` bits of the key, ascending; equal keys keep their input
 * order.  Bits above `bits` are carried but ignored for ordering.
 *   keys_in, vals_in    device [n], only read
 *   keys_out, vals_out  device [n], caller-allocated; must not alias the inputs
 *   n                   0 <= n < 2^31
 *   bits                1..64
 * Stream-ordered (no host synchronisation).  Uses the library's workspace.
 * Returns RS_OK, RS_EINVAL, RS_ENOMEM or RS_EDEVICE.
 */
int rs_sort_pairs_u64_i32(const uint64_t* keys_in, uint64_t* keys_out,
                          const int32_t* vals_in, int32_t* vals_out, int64_t n, int bits,
                          void* stream);

/*
 * Launch-shape tuning table (process-wide).  The batched form runs every
 * recursion level in size-bucketed kernels; these knobs pick among the
 * compiled launch shapes, and results are identical for every choice (only
 * speed changes).  Knobs:
 *   "small_threads_256"   threads per workgroup, nodes of 65..256 members:   128, 256
 *   "small_threads_1024"  threads per workgroup, nodes of 257..1024 members: 256, 512, 1024
 *   "small_threads_2048"  threads per workgroup, nodes of 1025..2048:        512, 1024
 *   "xcd_chunk"           longest run of consecutive 64-member tiles one XCD
 *                         takes in the large-node search kernels:           256, 1024, 4096
 * rs_tune_set: RS_OK, or RS_EINVAL for an unknown knob or a value not in its
 * list.  rs_tune_get: stores the current value, writes up to max_choices of
 * the allowed values into choices (host, may be NULL) and returns how many
 * there are, or RS_EINVAL.  rs_tune_name: name of knob `index` (0-based),
 * NULL past the last.  Not to be changed while a library call runs.
 */
int rs_tune_set(const char* knob, int value);
int rs_tune_get(const char* knob, int* value, int32_t* choices, int max_choices);
const char* rs_tune_name(int index);

/*
 * Releases the library's device workspaces on the current device.  The
 * library keeps grow-only workspaces between calls so repeated calls do not
 * allocate; a caller that needs the memory back (for example before working
 * on a 1024^3 result itself) calls this.  The next call allocates again.
 * Must not overlap a running library call on the same device.  Returns RS_OK
 * or RS_EDEVICE.
 */
int rs_release_workspace(void);

/* Releases an rs_tree* (struct and device arrays).  NULL is a no-op. */
void rs_free(void* p);

/* Static description of a status code. */
const char* rs_strerror(int status);

/* Library version string (static). */
const char* rs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RSFOF_H */
