// api.hip -- the extern "C" entry points: argument checks, then dispatch to
// the device pipelines.  No device work happens before the checks pass.
#include <math.h>
#include <stdlib.h>

#include "common.h"

namespace rs {
int fof3d_run(const float* x, const float* y, const float* z, int64_t n, float L, float ll,
              int32_t* labels, int64_t* n_groups, hipStream_t st);
int seeds_run(const float* x, const float* y, const float* z, const float* vx,
              const float* vy, const float* vz, int64_t n, float L, int64_t m, int64_t nlev,
              const int32_t* level, const int32_t* parent, const int32_t* min_index,
              const int32_t* size, const int32_t* deepest, const float* fa, const float* fc,
              const float* props, int32_t* halo, hipStream_t st);
int fof3d_noalloc_run(const float* x, const float* y, const float* z, int64_t n, float L,
                      float ll, int32_t* labels, int64_t* n_groups, hipStream_t st);
int fof3d_subbox_run(const float* x, const float* y, const float* z, int64_t n,
                     int64_t n_owned, const float* lo, const float* hi, float gw, float ll,
                     int32_t* labels, int32_t* ghost_links, int64_t* n_links, hipStream_t st);
int phase_run(const float* x, const float* y, const float* z, const float* vx,
              const float* vy, const float* vz, int64_t n, float L, const int32_t* labels,
              int32_t min_group, int32_t min_sub, double f, uint32_t flags, const void* model,
              rs_tree** out, hipStream_t st);
void tree_release(rs_tree* t);
int props_run(const float* x, const float* y, const float* z, const float* vx,
              const float* vy, const float* vz, int64_t n, float L, int64_t m, int64_t nlev,
              const int32_t* level, const int32_t* parent, const int32_t* min_index,
              const int32_t* size, const int32_t* deepest, float* props, hipStream_t st);

static int device_ready() {
    int cnt = 0;
    hipError_t e = hipGetDeviceCount(&cnt);
    if (e != hipSuccess || cnt < 1) {
        (void)hipGetLastError();
        return RS_EDEVICE;
    }
    return RS_OK;
}
}  // namespace rs

extern "C" {

int rs_fof3d(const float* x, const float* y, const float* z, int64_t n, float box,
             float link_len, int32_t* labels, int64_t* n_groups, void* stream) {
    if (n < 0 || n >= (int64_t)1 << 31) return RS_EINVAL;
    if (!(box > 0.0f) || !isfinite(box)) return RS_EINVAL;
    if (!(link_len > 0.0f) || !(link_len < 0.5f * box)) return RS_EINVAL;
    if (n > 0 && (!x || !y || !z || !labels)) return RS_EINVAL;
    RS_TRY(rs::device_ready());
    if (n == 0) {
        if (n_groups) *n_groups = 0;
        return RS_OK;
    }
    std::unique_lock<std::mutex> lk;
    RS_TRY(rs::call_lock(&lk));
    RS_TRY(rs::arena_call_begin(1u << rs::AR_BASE));
    return rs::fof3d_run(x, y, z, n, box, link_len, labels, n_groups,
                         static_cast<hipStream_t>(stream));
}

int rs_fof3d_noalloc(const float* x, const float* y, const float* z, int64_t n, float box,
                     float link_len, int32_t* labels, int64_t* n_groups, void* stream) {
    if (n < 0 || n >= (int64_t)1 << 31) return RS_EINVAL;
    if (!(box > 0.0f) || !isfinite(box)) return RS_EINVAL;
    if (!(link_len > 0.0f) || !(link_len < 0.5f * box)) return RS_EINVAL;
    if (n > 0 && (!x || !y || !z || !labels)) return RS_EINVAL;
    RS_TRY(rs::device_ready());
    if (n == 0) {
        if (n_groups) *n_groups = 0;
        return RS_OK;
    }
    std::unique_lock<std::mutex> lk;
    RS_TRY(rs::call_lock(&lk));
    return rs::fof3d_noalloc_run(x, y, z, n, box, link_len, labels, n_groups,
                                 static_cast<hipStream_t>(stream));
}

int rs_fof3d_subbox(const float* x, const float* y, const float* z, int64_t n, int64_t n_owned,
                    const float* lo, const float* hi, float ghost_width, float link_len,
                    int32_t* labels, int32_t* ghost_links, int64_t* n_links, void* stream) {
    if (n < 0 || n >= (int64_t)1 << 31 || n_owned < 0 || n_owned > n) return RS_EINVAL;
    if (!lo || !hi) return RS_EINVAL;
    for (int a = 0; a < 3; a++)
        if (!isfinite(lo[a]) || !isfinite(hi[a]) || !(hi[a] > lo[a])) return RS_EINVAL;
    if (!(ghost_width >= 0.0f) || !isfinite(ghost_width)) return RS_EINVAL;
    if (!(link_len > 0.0f) || !isfinite(link_len)) return RS_EINVAL;
    if (ghost_links && !n_links) return RS_EINVAL;
    if (n > 0 && (!x || !y || !z || !labels)) return RS_EINVAL;
    RS_TRY(rs::device_ready());
    if (n == 0) {
        if (n_links) *n_links = 0;
        return RS_OK;
    }
    std::unique_lock<std::mutex> lk;
    RS_TRY(rs::call_lock(&lk));
    RS_TRY(rs::arena_call_begin(1u << rs::AR_BASE));
    return rs::fof3d_subbox_run(x, y, z, n, n_owned, lo, hi, ghost_width, link_len, labels,
                                ghost_links, n_links, static_cast<hipStream_t>(stream));
}

int rs_phase_fof_batch(const float* x, const float* y, const float* z, const float* vx,
                       const float* vy, const float* vz, int64_t n, float box,
                       const int32_t* fof_labels, int32_t min_group, int32_t min_sub, double f,
                       uint32_t flags, const void* model, rs_tree** out, void* stream) {
    if (!out) return RS_EINVAL;
    if (n < 0 || n >= (int64_t)1 << 31) return RS_EINVAL;
    if (!(box > 0.0f) || !isfinite(box)) return RS_EINVAL;
    if (min_group < 2 || min_sub < 2) return RS_EINVAL;
    if (!(f > 0.0 && f <= 1.0)) return RS_EINVAL;
    if ((flags & ~(uint32_t)RS_FEATURES) > RS_LEARNED) return RS_EINVAL;
    if ((flags & 0xffu) == RS_LEARNED && !model) return RS_EINVAL;
    if (n > 0 && (!x || !y || !z || !vx || !vy || !vz || !fof_labels)) return RS_EINVAL;
    RS_TRY(rs::device_ready());
    std::unique_lock<std::mutex> lk;
    RS_TRY(rs::call_lock(&lk));
    RS_TRY(rs::arena_call_begin((1u << rs::AR_BASE) | (1u << rs::AR_LARGE) |
                                (1u << rs::AR_TREE) | (1u << rs::AR_MLP)));
    return rs::phase_run(x, y, z, vx, vy, vz, n, box, fof_labels, min_group, min_sub, f, flags,
                         model, out, static_cast<hipStream_t>(stream));
}

int rs_halo_props(const float* x, const float* y, const float* z, const float* vx,
                  const float* vy, const float* vz, int64_t n, float box, int64_t n_nodes,
                  int64_t n_levels, const int32_t* level, const int32_t* parent,
                  const int32_t* min_index, const int32_t* size, const int32_t* deepest,
                  float* props, void* stream) {
    if (n < 0 || n >= (int64_t)1 << 31) return RS_EINVAL;
    if (n_nodes < 0 || n_nodes >= (int64_t)1 << 31) return RS_EINVAL;
    if (n_levels < 0 || n_levels > n_nodes) return RS_EINVAL;
    if (n_nodes > 0 && n_levels < 1) return RS_EINVAL;
    if (!(box > 0.0f) || !(box < 2048.0f)) return RS_EINVAL;
    if (n > 0 && (!x || !y || !z || !vx || !vy || !vz || !deepest)) return RS_EINVAL;
    if (n_nodes > 0 && (!level || !parent || !min_index || !size || !props)) return RS_EINVAL;
    if (n == 0 && n_nodes > 0) return RS_EINVAL;   /* nodes without particles */
    RS_TRY(rs::device_ready());
    if (n == 0) return RS_OK;
    std::unique_lock<std::mutex> lk;
    RS_TRY(rs::call_lock(&lk));
    RS_TRY(rs::arena_call_begin(1u << rs::AR_BASE));
    return rs::props_run(x, y, z, vx, vy, vz, n, box, n_nodes, n_levels, level, parent,
                         min_index, size, deepest, props, static_cast<hipStream_t>(stream));
}

int rs_seed_assign(const float* x, const float* y, const float* z, const float* vx,
                   const float* vy, const float* vz, int64_t n, float box, int64_t n_nodes,
                   int64_t n_levels, const int32_t* level, const int32_t* parent,
                   const int32_t* min_index, const int32_t* size, const int32_t* deepest,
                   const float* a, const float* c, const float* props, int32_t* halo,
                   void* stream) {
    if (n < 0 || n >= (int64_t)1 << 31) return RS_EINVAL;
    if (n_nodes < 0 || n_nodes >= (int64_t)1 << 31) return RS_EINVAL;
    if (n_levels < 0 || n_levels > n_nodes) return RS_EINVAL;
    if (n_nodes > 0 && n_levels < 1) return RS_EINVAL;
    if (!(box > 0.0f) || !isfinite(box)) return RS_EINVAL;
    if (n > 0 && (!x || !y || !z || !vx || !vy || !vz || !deepest || !halo)) return RS_EINVAL;
    if (n_nodes > 0 && (!level || !parent || !min_index || !size || !a || !c || !props))
        return RS_EINVAL;
    if (n == 0 && n_nodes > 0) return RS_EINVAL;
    RS_TRY(rs::device_ready());
    if (n == 0) return RS_OK;
    std::unique_lock<std::mutex> lk;
    RS_TRY(rs::call_lock(&lk));
    RS_TRY(rs::arena_call_begin(1u << rs::AR_BASE));
    return rs::seeds_run(x, y, z, vx, vy, vz, n, box, n_nodes, n_levels, level, parent,
                         min_index, size, deepest, a, c, props, halo,
                         static_cast<hipStream_t>(stream));
}

int rs_sort_pairs_u64_i32(const uint64_t* keys_in, uint64_t* keys_out, const int32_t* vals_in,
                          int32_t* vals_out, int64_t n, int bits, void* stream) {
    if (n < 0 || n >= (int64_t)1 << 31 || bits < 1 || bits > 64) return RS_EINVAL;
    if (n > 0 && (!keys_in || !keys_out || !vals_in || !vals_out)) return RS_EINVAL;
    if (n > 0 && ((const void*)keys_in == (const void*)keys_out ||
                  (const void*)vals_in == (const void*)vals_out))
        return RS_EINVAL;
    RS_TRY(rs::device_ready());
    if (n == 0) return RS_OK;
    rs::Arena* ar = nullptr;
    const size_t tb = rs::sort_temp_bytes(n);
    std::unique_lock<std::mutex> lk;
    RS_TRY(rs::call_lock(&lk));
    RS_TRY(rs::arena_call_begin(1u << rs::AR_SORT));
    RS_TRY(rs::arena_reserve(rs::AR_SORT, tb, &ar));
    void* temp = rs::arena_take(ar, tb);
    if (!temp) return RS_EINTERNAL;
    return rs::sort_pairs_u64_i32(keys_in, keys_out, vals_in, vals_out, n, bits, temp, tb,
                                  static_cast<hipStream_t>(stream));
}

int rs_release_workspace(void) {
    RS_TRY(rs::device_ready());
    std::unique_lock<std::mutex> lk;
    RS_TRY(rs::call_lock(&lk));
    RS_HIP(hipDeviceSynchronize());
    for (int k = 0; k < rs::N_ARENAS; k++) RS_TRY(rs::arena_release(k));
    return RS_OK;
}

void rs_free(void* p) {
    if (!p) return;
    rs::tree_release(static_cast<rs_tree*>(p));
}

const char* rs_strerror(int status) {
    switch (status) {
        case RS_OK: return "success";
        case RS_EINVAL: return "invalid argument";
        case RS_ERANGE: return "coordinate out of range or not finite";
        case RS_ENOMEM: return "device memory allocation failed";
        case RS_EDEVICE: return "no usable HIP device or HIP runtime error";
        case RS_EINTERNAL: return "internal capacity or consistency failure";
        case RS_ENOTIMPL: return "mode not implemented";
        default: return "unknown status";
    }
}

const char* rs_version(void) { return "rsfof 0.1 (gfx950)"; }

}  // extern "C"
