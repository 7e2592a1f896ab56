// Internal interfaces between the C-ABI layer and the kernel launchers.
#pragma once

#include <string>
#include <vector>

#include "common.h"

namespace mg {

// Per-plane layout of the record buckets and the kernel each plane runs.
//   Buckets are (plane, uv tile) pairs.  A tile is T x T cells; a record
//   belongs to the tile holding its footprint's first cell (k_lo_u, k_lo_v).
//   Planes are gathered into groups: a maximal run of consecutive planes of
//   one support class above 16 forms one group, every other plane is a group
//   of its own.  The buckets of a group are numbered tile-major,
//     bucket = base + tile * grp_n + (plane - grp_first),
//   so the records of one tile in all the group's planes are contiguous and
//   the output-stationary kernels commit each tile's region once.
struct PlaneLayout {
    int32_t S;          // support of the plane
    int32_t T;          // tile side in cells (8, 16 or 32)
    int32_t log2T;
    int32_t ntu, ntv;   // tiles per axis
    int64_t base;       // first bucket of the plane's group
    int32_t cls;        // gridder class (see grid.hip)
    uint32_t tap_off;   // first element of the plane in the plan's (phase-major) table
    uint32_t src_off;   // first element of the plane in the caller's bank
    float tmax;         // largest |re|, |im| of the plane's taps (a separable
                        // weight, a product of two taps, is bounded by tmax^2)
    int32_t grp_first;  // first plane of the group
    int32_t grp_n;      // planes in the group
    int32_t grp_smax;   // largest support in the group
};

// Plane and tile of a bucket, given the layout of any plane of its group.
__host__ __device__ inline void bucket_plane_tile(const PlaneLayout &g, uint32_t bucket,
                                                  int *plane, uint32_t *tile) {
    const uint32_t local = bucket - (uint32_t)g.base;
    *plane = g.grp_first + (int)(local % (uint32_t)g.grp_n);
    *tile = local / (uint32_t)g.grp_n;
}

// One chunk: up to R records of one bucket, cell-sorted inside the chunk.
//   bbox: k_lo ranges of the chunk's records relative to the tile origin,
//   packed umin | umax << 8 | vmin << 16 | vmax << 24.
struct Chunk {
    uint32_t start;
    uint32_t len;
    uint32_t bucket;
    uint32_t bbox;
};

// A plan's device arrays are carved from one arena (caller workspace, a
// stream-ordered allocation, or the library's static scratch), at offsets
// computed on the host from the geometry and the record count alone
// (plan_arena_bytes).  The arena also holds the build's temporaries.
struct PlanState {
    DevGeom geom{};
    mg_kernel_kind kind = MG_KERNEL_SEPARABLE;
    mg_dtype tap_dtype = MG_F32;
    int32_t nplanes_eff = 1;          // 1 for separable
    int64_t nrec = 0;
    int64_t nbuckets = 0;
    int64_t max_chunks = 0;
    int64_t table_elems = 0;          // elements of one copy of the plan's tap table
    int32_t R = 1024;                 // records per chunk (max)
    std::vector<PlaneLayout> planes;  // host copy
    // device arrays (inside the arena)
    void *taps = nullptr;             // plan-owned copy of the table(s)
    size_t taps_bytes = 0;
    RecMeta *smeta = nullptr;         // [nrec + kRecPad] sorted (first nvalid valid)
    uint32_t *sperm = nullptr;        // [nrec + kRecPad] original record index
    Chunk *chunks = nullptr;          // [max_chunks]
    uint32_t *plane_cfirst = nullptr; // [nplanes_eff + 1] first chunk of each plane's group
    uint32_t *bucket_cfirst = nullptr; // [nbuckets + 1] first chunk of each bucket
    uint2 *units = nullptr;           // [max_chunks] units of the plane groups (see plan.hip)
    uint32_t *group_nunits = nullptr; // [nplanes_eff] unit count, at each group's first plane
    PlaneLayout *d_planes = nullptr;  // [nplanes_eff]
    int64_t *counters = nullptr;      // [0] skipped, [1] valid, [2] chunks, [3], [4] scratch
    // build temporaries (inside the arena, unused after the build)
    uint32_t *hist = nullptr, *bstart = nullptr, *cursor = nullptr;   // [nbuckets]
    uint2 *sums = nullptr;                                            // [nscan + 1]
    size_t bytes = 0;                 // arena bytes
};

// Per-call scratch of the gridders (grid.hip): sorted visibilities, each
// unit's fixed-point scale word, one work counter per plane.
struct GridScratch {
    float4 *svis = nullptr;      // [2 (nrec + kRecPad)]
    int32_t *uinfo = nullptr;    // [max_chunks]
    uint32_t *queues = nullptr;  // [nplanes_eff]
};

// Errors (thread-local message).
mg_status set_error(mg_status s, const std::string &msg);

// Host layout of a plan (planes, groups, buckets, chunk bound) from the
// descriptors; no device work (api.hip).
mg_status plan_prepare(PlanState &P, const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec);

// Arena bytes of a prepared plan, and the carving of an arena of that size
// (256-byte aligned base) into its arrays (plan.hip).
size_t plan_arena_bytes(const PlanState &P);
void plan_carve(PlanState &P, void *arena);

// Bytes of the per-call scratch of launch_grid / launch_degrid, and its
// carving (grid.hip, degrid.hip).
size_t grid_scratch_bytes(const PlanState &P);
size_t degrid_scratch_bytes(const PlanState &P);

// Build steps (plan.hip), on a carved plan.  All asynchronous on `stream`;
// nothing is allocated.
mg_status plan_build(PlanState &P, const void *uvw, mg_dtype uvw_dtype, hipStream_t stream);
mg_status launch_compute_indices(const DevGeom &g, int64_t nrec, const void *uvw,
                                 mg_dtype uvw_dtype, int32_t *k_lo_u, int32_t *k_lo_v,
                                 int32_t *o_u, int32_t *o_v, int32_t *plane, uint8_t *valid,
                                 int64_t *d_nskipped, hipStream_t stream);

// Uploads the plane layouts and lays out the plan's tap table (table_elems
// elements per copy) from the caller's bank at src, followed for
// W-projection by its complex conjugate (plan.hip).
mg_status plan_taps(PlanState &P, const void *src, int64_t table_elems, hipStream_t stream);

// Hot kernels (grid.hip, degrid.hip).  `scratch` holds grid_scratch_bytes /
// degrid_scratch_bytes (256-byte aligned); nullptr: allocated and released
// stream-ordered inside the call.
mg_status launch_grid(const PlanState &P, const void *vis, void *grid, void *scratch,
                      hipStream_t stream);
mg_status launch_degrid(const PlanState &P, const void *grid, void *vis_out, void *scratch,
                        hipStream_t stream);

// Stream-ordered scratch from the library's memory pool of the current
// device, which keeps up to kPoolKeepBytes of freed memory cached between
// calls (the device's default pool returns it at every synchronisation,
// which made one-shot calls after a synchronisation pay for mapping their
// scratch again) (api.hip).
constexpr uint64_t kPoolKeepBytes = uint64_t(8) << 30;
hipError_t scratch_alloc(void **p, size_t bytes, hipStream_t stream);
hipError_t scratch_free(void *p, hipStream_t stream);

// mg_grid with the plan and scratch in a caller-held arena that grows (in
// `stream`'s order, never shrinking) when a call needs more: the serving
// streams each keep one, so jobs allocate nothing once the arenas have grown
// (api.hip).
mg_status grid_in_arena(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec,
                        const void *uvw, mg_dtype uvw_dtype, const void *vis, void *grid,
                        void **arena, size_t *arena_bytes, hipStream_t stream);

// Workgroups of `kernel` (threads per workgroup, dynamic LDS bytes) that fit
// on the current device at once; device attributes and occupancy are queried
// once per (device, kernel, threads, lds) and cached (api.hip).
int resident_groups(const void *kernel, int threads, size_t lds);
int device_cus();
int device_lds_limit();

// Bytes rounded up to the arena alignment.
constexpr size_t kArenaAlign = 256;
inline size_t arena_round(size_t b) { return (b + kArenaAlign - 1) & ~(kArenaAlign - 1); }

// Support classes (each has its own gridding and degridding kernels):
//   class 0: S <= 8   moving window, one slot per lane
//   class 1: S <= 16  moving window, up to 4 slots per lane
//   class 2: S <= 32  moving window held by teams of 2 waves, up to 8 slots
//                     per lane
//   class 3: S <= 64  blocked output-stationary kernel (registers per 8 x 8
//                     block of the unit's region)
// Classes 0-2 accumulate committed sums in a fixed-point LDS region (see
// grid.hip); class 3 commits its registers to the grid once per unit.
// Entries of padding after the sorted record arrays (metadata, and the
// gridder's sorted visibilities): the gridders load records in batches of
// two, one batch ahead, so their reads reach 3 entries past the last record
// of a range.
constexpr int kRecPad = 4;

inline size_t dtype_size(mg_dtype d) {
    switch (d) {
    case MG_F32: return 4;
    case MG_F64: return 8;
    case MG_F16: return 2;
    case MG_BF16: return 2;
    }
    return 0;
}

inline int support_class(int S) { return S <= 8 ? 0 : S <= 16 ? 1 : S <= 32 ? 2 : 3; }

}  // namespace mg
