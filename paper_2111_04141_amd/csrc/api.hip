// C ABI of the migrid library: argument checking, plan layout, one-shot calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

struct mg_plan {
    mg::PlanState st;
    hipEvent_t ready = nullptr;   // recorded after the build work
    void *owned = nullptr;        // arena allocated by the library (no caller workspace)
    hipStream_t create_stream = nullptr;
    // library-owned arenas only: the last call of the plan on each stream,
    // waited for before the arena is released
    std::mutex mu;
    std::vector<std::pair<hipStream_t, hipEvent_t>> uses;
};

namespace mg {

namespace {
thread_local std::string g_err;

int ilog2(int x) {
    int l = 0;
    while ((1 << (l + 1)) <= x) ++l;
    return l;
}

// Tile side for a gridder class: 16, or 8 where the LDS region
// (tile + S_max - 1)^2 x npol x 8 bytes would not fit the per-workgroup LDS
// limit.  Small tiles keep the region small, so several workgroups share a
// CU; the record density of all but the sparsest planes keeps the per-chunk
// region flush small next to the chunk's work.
int tile_for_class(int cls, int npol, int lds_limit) {
    (void)npol;
    if (cls == 3) return 16;
    const int smax = cls == 0 ? 8 : cls == 1 ? 16 : 32;
    // region: 8 int32 per cell (4 polarisations, re and im); keep room for
    // two workgroups per CU
    for (int T : {16, 8}) {
        size_t bytes = (size_t)(T + smax - 1) * (T + smax - 1) * 8 * sizeof(int32_t);
        if (2 * bytes <= (size_t)lds_limit) return T;
    }
    return 8;
}

mg_status check_common(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec,
                       const void *uvw, mg_dtype uvw_dtype) {
    if (!g || !k) return set_error(MG_EINVAL, "null descriptor");
    if (g->nu < 1 || g->nv < 1 || g->nu > kMaxN || g->nv > kMaxN)
        return set_error(MG_EINVAL, "grid size must be in [1, 65535]");
    if (g->npol < 1 || g->npol > 4) return set_error(MG_EINVAL, "npol must be in 1..4");
    if (g->beta < 1 || g->beta > kMaxBeta) return set_error(MG_EINVAL, "beta must be in 1..256");
    if (!std::isfinite(g->scale_u) || !std::isfinite(g->scale_v))
        return set_error(MG_EINVAL, "scale must be finite");
    if (nrec < 0 || nrec > 0x7ffffffeLL) return set_error(MG_EINVAL, "nrec must be in [0, 2^31-2]");
    if (nrec > 0 && !uvw) return set_error(MG_EINVAL, "null uvw");
    if (uvw_dtype != MG_F32 && uvw_dtype != MG_F64)
        return set_error(MG_EINVAL, "uvw dtype must be MG_F32 or MG_F64");
    if (k->tap_dtype != MG_F32 && k->tap_dtype != MG_F16 && k->tap_dtype != MG_BF16)
        return set_error(MG_EINVAL, "tap dtype must be MG_F32, MG_F16 or MG_BF16");
    if (!k->taps) return set_error(MG_EINVAL, "null taps");
    if (k->kind == MG_KERNEL_SEPARABLE || k->kind == MG_KERNEL_WSTACK) {
        if (k->kind == MG_KERNEL_WSTACK) {
            if (k->nplanes < 1 || k->nplanes > kMaxPlanes)
                return set_error(MG_EINVAL, "W-stacking layers must be in 1..128");
            if ((int64_t)k->nplanes * g->nv > kMaxN)
                return set_error(MG_EINVAL, "layers x nv must be at most 65535");
            if (!std::isfinite(k->inv_dw) || k->inv_dw < 0)
                return set_error(MG_EINVAL, "inv_dw must be finite and >= 0");
        }
        if (k->support < 1 || k->support > kMaxSupport)
            return set_error(MG_EINVAL, "support must be in 1..64");
        if (((int64_t)g->beta * k->support) % 2)
            return set_error(MG_EINVAL, "beta * support must be even");
        if (k->ntaps < (int64_t)g->beta * k->support + 1)
            return set_error(MG_EINVAL, "separable table shorter than beta*S+1");
        if (k->ntaps > 0x7fffffffLL) return set_error(MG_EINVAL, "tap table too large");
    } else if (k->kind == MG_KERNEL_WPROJ) {
        if (k->nplanes < 1 || k->nplanes > kMaxPlanes)
            return set_error(MG_EINVAL, "nplanes must be in 1..128");
        if (!k->plane_support || !k->plane_offset)
            return set_error(MG_EINVAL, "null plane_support / plane_offset");
        if (!std::isfinite(k->inv_dw) || k->inv_dw < 0)
            return set_error(MG_EINVAL, "inv_dw must be finite and >= 0");
        for (int p = 0; p < k->nplanes; ++p) {
            const int S = k->plane_support[p];
            if (S < 1 || S > kMaxSupport) return set_error(MG_EINVAL, "plane support must be in 1..64");
            if (((int64_t)g->beta * S) % 2) return set_error(MG_EINVAL, "beta * S_p must be even");
            const int64_t w = (int64_t)g->beta * S + 1;
            if (k->plane_offset[p] < 0 || k->plane_offset[p] + w * w > k->ntaps)
                return set_error(MG_EINVAL, "plane table outside the tap array");
            if (k->plane_offset[p] + w * w > (1LL << 30))
                return set_error(MG_EINVAL, "tap table too large (at most 2^30 complex taps)");
        }
    } else {
        return set_error(MG_EINVAL, "unknown kernel kind");
    }
    return MG_OK;
}

DevGeom make_geom(const mg_grid_desc *g, const mg_kernel_desc *k) {
    DevGeom d;
    std::memset(&d, 0, sizeof d);
    d.nu = g->nu;
    d.nv = g->nv;
    d.npol = g->npol;
    d.beta = g->beta;
    d.scale_u = g->scale_u;
    d.scale_v = g->scale_v;
    if (k->kind == MG_KERNEL_WPROJ) {
        d.nplanes = k->nplanes;
        d.support = 0;
        d.inv_dw = k->inv_dw;
        d.conj_base = k->ntaps;
        for (int p = 0; p < k->nplanes; ++p) {
            d.plane_support[p] = k->plane_support[p];
            d.plane_offset[p] = k->plane_offset[p];
        }
    } else {
        d.nplanes = 0;
        d.support = k->support;
        d.plane_support[0] = k->support;
        d.plane_offset[0] = 0;
        if (k->kind == MG_KERNEL_WSTACK) {
            // the layers' grids stacked along v: one tall separable grid
            d.layers = k->nplanes;
            d.layer_nv = g->nv;
            d.nv = k->nplanes * g->nv;
            d.inv_dw = k->inv_dw;
        }
    }
    return d;
}

// Records the plan's use on `stream` (library-owned arenas only).
void note_use(mg_plan *p, hipStream_t stream) {
    if (!p->owned) return;
    std::lock_guard<std::mutex> lk(p->mu);
    for (auto &u : p->uses) {
        if (u.first == stream) {
            hipEventRecord(u.second, stream);
            return;
        }
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
        hipEventRecord(ev, stream);
        p->uses.emplace_back(stream, ev);
    }
}

// Lays out the plan in `arena` (plan_arena_bytes(P) bytes) and queues its
// build on `stream`.
mg_status build_in(PlanState &P, const mg_kernel_desc *k, const void *uvw, mg_dtype uvw_dtype,
                   void *arena, hipStream_t stream) {
    plan_carve(P, arena);
    const mg_status st = plan_taps(P, k->taps, P.table_elems, stream);
    if (st != MG_OK) return st;
    return plan_build(P, uvw, uvw_dtype, stream);
}

__global__ void add_count_kernel(const int64_t *src, int64_t *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst += *src;
}

}  // namespace

mg_status set_error(mg_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

// Device queries, once per device (and per kernel configuration for the
// occupancy): launches on the serving path must not pay for them each time.
namespace {
std::mutex g_dev_mu;
std::map<int, std::pair<int, int>> g_dev_attr;   // device -> (CUs, LDS per workgroup)
std::map<std::tuple<int, const void *, int, size_t>, int> g_occ;

std::pair<int, int> dev_attr(int *dev_out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (dev_out) *dev_out = dev;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_dev_attr.find(dev);
    if (it != g_dev_attr.end()) return it->second;
    int cus = 0, lds = 0;
    const bool ok =
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        cus > 0 && lds > 0;
    if (!ok) return {1, 65536};   // no device: host-only size queries (not cached)
    return g_dev_attr[dev] = {cus, lds};
}
}  // namespace

namespace {
std::map<int, hipMemPool_t> g_pools;   // device -> the library's pool
}  // namespace

hipError_t scratch_alloc(void **p, size_t bytes, hipStream_t stream) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    hipMemPool_t pool = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_dev_mu);
        auto it = g_pools.find(dev);
        if (it != g_pools.end()) {
            pool = it->second;
        } else {
            hipMemPoolProps props;
            std::memset(&props, 0, sizeof props);
            props.allocType = hipMemAllocationTypePinned;
            props.location.type = hipMemLocationTypeDevice;
            props.location.id = dev;
            e = hipMemPoolCreate(&pool, &props);
            if (e != hipSuccess) return e;
            uint64_t keep = kPoolKeepBytes;
            hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
            // a block freed on one stream must not be handed to another
            // stream by making that stream wait for the first: concurrent
            // callers (the server's job streams) would be chained together
            int no = 0;
            hipMemPoolSetAttribute(pool, hipMemPoolReuseAllowInternalDependencies, &no);
            g_pools[dev] = pool;
        }
    }
    return hipMallocFromPoolAsync(p, bytes, pool, stream);
}

hipError_t scratch_free(void *p, hipStream_t stream) { return hipFreeAsync(p, stream); }

int device_cus() { return dev_attr(nullptr).first; }
int device_lds_limit() { return dev_attr(nullptr).second; }

int resident_groups(const void *kernel, int threads, size_t lds) {
    int dev = 0;
    const int cus = dev_attr(&dev).first;
    const auto key = std::make_tuple(dev, kernel, threads, lds);
    {
        std::lock_guard<std::mutex> lk(g_dev_mu);
        auto it = g_occ.find(key);
        if (it != g_occ.end()) return it->second;
    }
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, lds) != hipSuccess ||
        per < 1)
        per = 1;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    return g_occ[key] = per * cus;
}

// Host layout of a plan: planes, support classes, tiles, plane groups and
// their buckets, the chunk bound and the tap table's size.
mg_status plan_prepare(PlanState &P, const mg_grid_desc *g, const mg_kernel_desc *k,
                       int64_t nrec) {
    P.geom = make_geom(g, k);
    // W-stacking grids like a separable kernel on the stacked layer grids
    P.kind = k->kind == MG_KERNEL_WSTACK ? MG_KERNEL_SEPARABLE : k->kind;
    P.tap_dtype = k->tap_dtype;
    P.nrec = nrec;
    P.nplanes_eff = (k->kind == MG_KERNEL_WPROJ) ? k->nplanes : 1;
    // chunk size: enough chunks to fill the chip, at most 2048 records
    int64_t R = nrec / 4096;
    P.R = (int32_t)std::max<int64_t>(64, std::min<int64_t>(2048, R));
    const int lds = device_lds_limit();
    P.planes.resize(P.nplanes_eff);
    for (int p = 0; p < P.nplanes_eff; ++p) {
        PlaneLayout &L = P.planes[p];
        L.S = (k->kind == MG_KERNEL_WPROJ) ? k->plane_support[p] : k->support;
        L.cls = support_class(L.S);
        L.T = tile_for_class(L.cls, g->npol, lds);
        L.log2T = ilog2(L.T);
        L.ntu = (P.geom.nu + L.T - 1) / L.T;
        L.ntv = (P.geom.nv + L.T - 1) / L.T;
        L.tmax = 0.0f;   // raised on the device by the tap layout
    }
    // the plan's tap table: planes one after another, phase-major
    int64_t table = 0;
    for (int p = 0; p < P.nplanes_eff; ++p) {
        PlaneLayout &L = P.planes[p];
        const int64_t w = (int64_t)g->beta * L.S;   // entries per axis
        L.tap_off = (uint32_t)table;
        L.src_off = (k->kind == MG_KERNEL_WPROJ) ? (uint32_t)k->plane_offset[p] : 0u;
        P.geom.plane_offset[p] = table;
        table += (k->kind == MG_KERNEL_WPROJ) ? w * w : w;
    }
    P.geom.conj_base = table;
    if (table >= (1LL << 30)) return set_error(MG_EUNSUPPORTED, "tap table too large");
    P.table_elems = table;
    const bool wproj = k->kind == MG_KERNEL_WPROJ;
    P.taps_bytes = dtype_size(k->tap_dtype) * (wproj ? 2 : 1) * (size_t)table * (wproj ? 2 : 1);
    // groups: runs of consecutive planes of one class share their buckets,
    // numbered tile-major
    int64_t base = 0;
    for (int p0 = 0; p0 < P.nplanes_eff;) {
        int p1 = p0 + 1;
        while (p1 < P.nplanes_eff && P.planes[p1].cls == P.planes[p0].cls) ++p1;
        int smax = 0;
        for (int p = p0; p < p1; ++p) smax = std::max(smax, P.planes[p].S);
        for (int p = p0; p < p1; ++p) {
            PlaneLayout &L = P.planes[p];
            L.base = base;
            L.grp_first = p0;
            L.grp_n = p1 - p0;
            L.grp_smax = smax;
        }
        base += (int64_t)P.planes[p0].ntu * P.planes[p0].ntv * (p1 - p0);
        p0 = p1;
    }
    P.nbuckets = base;
    if (base >= 0x7fffffffLL) return set_error(MG_EUNSUPPORTED, "too many (plane, tile) buckets");
    P.max_chunks = base + nrec / P.R + 1;
    return MG_OK;
}

}  // namespace mg

using namespace mg;

extern "C" {

const char *mg_status_str(mg_status s) {
    switch (s) {
    case MG_OK: return "ok";
    case MG_EINVAL: return "invalid argument";
    case MG_ENOMEM: return "out of memory";
    case MG_EDEVICE: return "device error";
    case MG_EUNSUPPORTED: return "unsupported";
    case MG_EBUSY: return "busy";
    }
    return "unknown status";
}

const char *mg_last_error(void) { return g_err.c_str(); }

mg_status mg_compute_indices(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec,
                             const void *uvw, mg_dtype uvw_dtype, int32_t *k_lo_u,
                             int32_t *k_lo_v, int32_t *o_u, int32_t *o_v, int32_t *plane,
                             uint8_t *valid, int64_t *d_nskipped, hipStream_t stream) {
    mg_status s = check_common(g, k, nrec, uvw, uvw_dtype);
    if (s != MG_OK) return s;
    if (nrec > 0 && (!k_lo_u || !k_lo_v || !o_u || !o_v || !plane || !valid))
        return set_error(MG_EINVAL, "null output array");
    return launch_compute_indices(make_geom(g, k), nrec, uvw, uvw_dtype, k_lo_u, k_lo_v, o_u, o_v,
                                  plane, valid, d_nskipped, stream);
}

mg_status mg_plan_workspace_size(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec,
                                 size_t *bytes) {
    if (!bytes) return set_error(MG_EINVAL, "null bytes output");
    *bytes = 0;
    // the uvw pointer is not needed for the size: check the rest
    mg_status s = check_common(g, k, nrec, reinterpret_cast<const void *>(1), MG_F32);
    if (s != MG_OK) return s;
    PlanState P;
    s = plan_prepare(P, g, k, nrec);
    if (s != MG_OK) return s;
    *bytes = plan_arena_bytes(P);
    return MG_OK;
}

mg_status mg_plan_create(mg_plan **plan, const mg_grid_desc *g, const mg_kernel_desc *k,
                         int64_t nrec, const void *uvw, mg_dtype uvw_dtype, void *workspace,
                         hipStream_t stream) {
    if (!plan) return set_error(MG_EINVAL, "null plan output");
    *plan = nullptr;
    mg_status s = check_common(g, k, nrec, uvw, uvw_dtype);
    if (s != MG_OK) return s;
    if (workspace && (reinterpret_cast<uintptr_t>(workspace) % kArenaAlign) != 0)
        return set_error(MG_EINVAL, "workspace must be 256-byte aligned");
    mg_plan *p = new (std::nothrow) mg_plan;
    if (!p) return set_error(MG_ENOMEM, "host allocation failed");
    p->create_stream = stream;
    s = plan_prepare(p->st, g, k, nrec);
    void *arena = workspace;
    if (s == MG_OK && !arena) {
        const size_t bytes = plan_arena_bytes(p->st);
        hipError_t e = scratch_alloc(&arena, std::max<size_t>(bytes, kArenaAlign), stream);
        if (e != hipSuccess) {
            arena = nullptr;
            s = set_error(MG_ENOMEM, std::string("plan allocation: ") + hipGetErrorString(e));
        }
        p->owned = arena;
    }
    if (s == MG_OK) s = build_in(p->st, k, uvw, uvw_dtype, arena, stream);
    if (s == MG_OK) {
        if (hipEventCreateWithFlags(&p->ready, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(p->ready, stream) != hipSuccess)
            s = set_error(MG_EDEVICE, "event record failed");
    }
    if (s != MG_OK) {
        if (p->owned) scratch_free(p->owned, stream);
        if (p->ready) hipEventDestroy(p->ready);
        delete p;
        return s;
    }
    *plan = p;
    return MG_OK;
}

mg_status mg_plan_grid(const mg_plan *plan, const void *vis, void *grid, hipStream_t stream) {
    if (!plan) return set_error(MG_EINVAL, "null plan");
    if (plan->st.nrec > 0 && !vis) return set_error(MG_EINVAL, "null vis");
    if (!grid) return set_error(MG_EINVAL, "null grid");
    const mg_status s = launch_grid(plan->st, vis, grid, nullptr, stream);
    note_use(const_cast<mg_plan *>(plan), stream);
    return s;
}

mg_status mg_plan_degrid(const mg_plan *plan, const void *grid, void *vis_out,
                         hipStream_t stream) {
    if (!plan) return set_error(MG_EINVAL, "null plan");
    if (!grid) return set_error(MG_EINVAL, "null grid");
    if (plan->st.nrec > 0 && !vis_out) return set_error(MG_EINVAL, "null vis_out");
    const mg_status s = launch_degrid(plan->st, grid, vis_out, nullptr, stream);
    note_use(const_cast<mg_plan *>(plan), stream);
    return s;
}

mg_status mg_plan_nskipped(const mg_plan *plan, int64_t *nskipped) {
    if (!plan || !nskipped) return set_error(MG_EINVAL, "null argument");
    if (hipEventSynchronize(plan->ready) != hipSuccess) return set_error(MG_EDEVICE, "event sync failed");
    int64_t v = 0;
    if (hipMemcpy(&v, plan->st.counters, sizeof v, hipMemcpyDeviceToHost) != hipSuccess)
        return set_error(MG_EDEVICE, "counter copy failed");
    *nskipped = v;
    return MG_OK;
}

mg_status mg_plan_bytes(const mg_plan *plan, size_t *bytes) {
    if (!plan || !bytes) return set_error(MG_EINVAL, "null argument");
    *bytes = plan->st.bytes;
    return MG_OK;
}

mg_status mg_plan_destroy(mg_plan *plan) {
    if (!plan) return MG_OK;
    mg_status s = MG_OK;
    if (plan->owned) {
        // the library's arena: released stream-ordered after the build and
        // after the plan's last call on every stream it was used on (no
        // host or device-wide wait)
        hipStream_t st = plan->create_stream;
        for (auto &u : plan->uses)
            if (hipStreamWaitEvent(st, u.second, 0) != hipSuccess) s = MG_EDEVICE;
        if (scratch_free(plan->owned, st) != hipSuccess) {
            hipEventSynchronize(plan->ready);
            for (auto &u : plan->uses) hipEventSynchronize(u.second);
            hipFree(plan->owned);
        }
    }
    for (auto &u : plan->uses) hipEventDestroy(u.second);
    if (plan->ready) hipEventDestroy(plan->ready);
    delete plan;
    return s == MG_OK ? MG_OK : set_error(s, "stream wait failed");
}

}  // extern "C"

// Static scratch of mg_grid_static: the plan and the gridding scratch of
// one call, for callers that cannot allocate device memory.  Every GPU the
// library runs on holds its own copy until the process ends.  In host code
// the array's name is not a device address: its address on each device is
// queried once, with that device current, and kept.
static constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

extern "C" {

namespace {
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;   // device -> address of its copy

mg_status static_scratch(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(MG_EDEVICE, "no device");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return MG_OK;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return set_error(MG_EDEVICE, std::string("static scratch address: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
    *out = ptr;
    return MG_OK;
}

// One-shot calls: plan and call scratch in one stream-ordered allocation.
// The one-shot pipeline (index, sort, gather, grid or degrid) in `arena`,
// which holds at least plan_arena_bytes + the call's scratch bytes; with a
// null arena the bytes come from the library's pool for this call.
mg_status one_shot(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec,
                   const void *uvw, mg_dtype uvw_dtype, bool gridding, const void *in, void *out,
                   int64_t *d_nskipped, hipStream_t stream, void *arena = nullptr) {
    PlanState P;
    mg_status s = plan_prepare(P, g, k, nrec);
    if (s != MG_OK) return s;
    const size_t pb = plan_arena_bytes(P);
    const size_t cb = gridding ? grid_scratch_bytes(P) : degrid_scratch_bytes(P);
    void *own = nullptr;
    if (!arena) {
        hipError_t e = scratch_alloc(&own, pb + cb, stream);
        if (e != hipSuccess) return set_error(MG_ENOMEM, std::string("scratch allocation: ") + hipGetErrorString(e));
        arena = own;
    }
    s = build_in(P, k, uvw, uvw_dtype, arena, stream);
    void *scratch = static_cast<char *>(arena) + pb;
    if (s == MG_OK)
        s = gridding ? launch_grid(P, in, out, scratch, stream)
                     : launch_degrid(P, in, out, scratch, stream);
    if (s == MG_OK && d_nskipped)
        hipLaunchKernelGGL(add_count_kernel, dim3(1), dim3(64), 0, stream, P.counters, d_nskipped);
    if (own) scratch_free(own, stream);
    return s;
}
}  // namespace


mg_status mg_grid(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec, const void *uvw,
                  mg_dtype uvw_dtype, const void *vis, void *grid, int64_t *d_nskipped,
                  hipStream_t stream) {
    mg_status s = check_common(g, k, nrec, uvw, uvw_dtype);
    if (s != MG_OK) return s;
    if (nrec > 0 && !vis) return set_error(MG_EINVAL, "null vis");
    if (!grid) return set_error(MG_EINVAL, "null grid");
    return one_shot(g, k, nrec, uvw, uvw_dtype, true, vis, grid, d_nskipped, stream);
}

mg_status mg_grid_static(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec,
                         const void *uvw, mg_dtype uvw_dtype, const void *vis, void *grid,
                         int64_t *d_nskipped, hipStream_t stream) {
    mg_status s = check_common(g, k, nrec, uvw, uvw_dtype);
    if (s != MG_OK) return s;
    if (nrec > 0 && !vis) return set_error(MG_EINVAL, "null vis");
    if (!grid) return set_error(MG_EINVAL, "null grid");
    PlanState P;
    s = plan_prepare(P, g, k, nrec);
    if (s != MG_OK) return s;
    const size_t pb = plan_arena_bytes(P);
    const size_t need = pb + grid_scratch_bytes(P);
    if (need > kStaticScratchBytes)
        return set_error(MG_ENOMEM, "mg_grid_static needs " + std::to_string(need) +
                                        " bytes of scratch; the static scratch holds " +
                                        std::to_string(kStaticScratchBytes));
    void *arena = nullptr;
    s = static_scratch(&arena);
    if (s != MG_OK) return s;
    s = build_in(P, k, uvw, uvw_dtype, arena, stream);
    if (s == MG_OK) s = launch_grid(P, vis, grid, static_cast<char *>(arena) + pb, stream);
    if (s == MG_OK && d_nskipped)
        hipLaunchKernelGGL(add_count_kernel, dim3(1), dim3(64), 0, stream, P.counters, d_nskipped);
    if (s == MG_OK && hipGetLastError() != hipSuccess) s = set_error(MG_EDEVICE, "launch failed");
    return s;
}

size_t mg_grid_static_capacity(void) { return kStaticScratchBytes; }

mg_status mg_degrid(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec,
                    const void *uvw, mg_dtype uvw_dtype, const void *grid, void *vis_out,
                    int64_t *d_nskipped, hipStream_t stream) {
    mg_status s = check_common(g, k, nrec, uvw, uvw_dtype);
    if (s != MG_OK) return s;
    if (!grid) return set_error(MG_EINVAL, "null grid");
    if (nrec > 0 && !vis_out) return set_error(MG_EINVAL, "null vis_out");
    return one_shot(g, k, nrec, uvw, uvw_dtype, false, grid, vis_out, d_nskipped, stream);
}

}  // extern "C"

mg_status mg::grid_in_arena(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec,
                        const void *uvw, mg_dtype uvw_dtype, const void *vis, void *grid,
                        void **arena, size_t *arena_bytes, hipStream_t stream) {
    mg_status s = check_common(g, k, nrec, uvw, uvw_dtype);
    if (s != MG_OK) return s;
    if (nrec > 0 && !vis) return set_error(MG_EINVAL, "null vis");
    if (!grid) return set_error(MG_EINVAL, "null grid");
    PlanState P;
    s = plan_prepare(P, g, k, nrec);
    if (s != MG_OK) return s;
    const size_t need = plan_arena_bytes(P) + grid_scratch_bytes(P);
    if (need > *arena_bytes) {
        // grow by at least half, in the stream's order: the old arena is
        // released after the stream's earlier work
        const size_t cap = std::max(need, *arena_bytes + *arena_bytes / 2);
        void *p = nullptr;
        const hipError_t e = scratch_alloc(&p, cap, stream);
        if (e != hipSuccess) return set_error(MG_ENOMEM, std::string("scratch allocation: ") + hipGetErrorString(e));
        if (*arena) scratch_free(*arena, stream);
        *arena = p;
        *arena_bytes = cap;
    }
    return one_shot(g, k, nrec, uvw, uvw_dtype, true, vis, grid, nullptr, stream, *arena);
}
