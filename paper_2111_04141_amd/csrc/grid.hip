// Gridding (scatter) kernels.
//
// Work unit: a run of chunks (up to R records each) of one uv tile over the
// planes of a group (consecutive planes of one support class), taken by one
// workgroup; units are handed out through a per-launch counter.
//
// Supports up to 32: moving window (grid_window_kernel).
//  * Each wave keeps a moving window of slots in registers: slot (su, sv)
//    owns the grid cells congruent to (su, sv) modulo S, so every record's
//    S x S footprint holds exactly one cell of each slot, and a slot's
//    accumulators (4 polarisations, complex) keep summing while its cell
//    stays inside the footprints of consecutive records.  This is the
//    owner-computes scheme of Romein's GPU gridder, which the thesis's
//    Convolutional Gridder builds on (Chapter 4); the slots are spread over
//    the 64 lanes of a wave (up to S = 16) or of a team of two waves (up to
//    S = 32), and the records come cell-sorted, so windows move rarely where
//    records are dense.
//  * When a slot's cell leaves the footprint its sums are committed into an
//    LDS copy of the unit's grid region (bounding box plus S-1 halo) shared
//    by the workgroup.  The region holds 32-bit fixed point: the gather
//    (gather_units_kernel) bounds every partial sum a unit can produce,
//    B = 2 * sum over its records of max|tap component of the record's
//    plane| * max|visibility component|, picks the power-of-two scale 2^e
//    that maps B to at most 2^30, and stores the unit's visibilities already
//    multiplied by 2^e (exact), so the accumulators hold fixed-point units
//    and a commit is one conversion, rounded to nearest, and one integer LDS
//    atomic per component (integer LDS atomics run at full wave rate, unlike
//    float LDS atomics, which serialise per lane).  The sums cannot overflow
//    and each commit is off by at most half a quantum 2^-e, which is below
//    2^-30 B (2^e is the largest power of two with 2^e B <= 2^30).  At the end
//    of the unit the region is converted back to FP32 (times 2^-e) and added
//    to the grid with float atomics, one per touched cell.
//
// Supports above 32: blocked output-stationary kernel (grid_block_kernel),
// for the sparse planes of large |w|; see the kernel's comment.
//
// All polarisations are handled per visit: one tap load feeds 4 complex
// multiply-adds (the thesis's Polarisation Gain, Section 3.5).  Records are
// read on the scalar unit (visibilities become SGPR operands of the FMAs),
// and each carries the table offset of its first tap (in the conjugated copy
// of the bank for w < 0), so the per-record scalar work is small.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <type_traits>

#include "internal.h"

namespace mg {

namespace {

constexpr uint32_t kNoCell = 0xffffffffu;
constexpr int kBatch = 2;   // records per batch of scalar loads
// the last batch of a range starts at most kBatch - 1 past its end and the
// read-ahead batch kBatch further: the sorted arrays are padded for that
static_assert(2 * kBatch - 1 <= kRecPad, "record read-ahead runs past the padding");

// Waits for every outstanding scalar load.  Called once after a record
// loop's first batch is issued: otherwise the compiler places the wait for
// that batch at the loop top, where (scalar loads complete out of order) it
// also waits for the next batch's loads on every iteration.
__device__ inline void wait_scalar_loads() { __builtin_amdgcn_s_waitcnt(0xC07F); }


// Nearest integer (halves round up) in one instruction: the fixed-point
// commit of an accumulator that is already in units of the quantum.
__device__ inline int32_t round_to_fixed(float x) {
    int32_t r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// Per-unit word written by the gather: bits 0-7 the fixed-point exponent e
// plus 128 (the unit's visibilities are stored times 2^e), bit 8 set if the
// unit commits in fixed point, bit 9 set if one of its visibilities is not
// finite.
constexpr int32_t kUnitFixed = 1 << 8;
constexpr int32_t kUnitNonFinite = 1 << 9;
__device__ inline int unit_scale(int32_t info) { return (info & 0xff) - 128; }

struct GridParams {
    int32_t npol, nu, nv, beta;
    int32_t p_lo, p_hi;       // planes handled by this launch
};

// Two 16-bit lanes of a 32-bit word (packed 16-bit integer arithmetic).
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
__device__ inline u16x2 as_u16x2(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ inline uint32_t as_u32(u16x2 x) { return __builtin_bit_cast(uint32_t, x); }
// a.u b.u + a.v b.v + c (modulo 2^32) in one instruction, for a and b holding
// (u, v) in their 16-bit halves
__device__ inline uint32_t dot_uv(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_udot2(as_u16x2(a), as_u16x2(b), c, false);
}

// Visibilities of one record, 4 polarisations.
struct RecVis {
    float vr[4], vi[4];
};

__device__ inline RecVis unpack_vis(const float4 v01, const float4 v23) {
    RecVis f;
    f.vr[0] = v01.x; f.vi[0] = v01.y; f.vr[1] = v01.z; f.vi[1] = v01.w;
    f.vr[2] = v23.x; f.vi[2] = v23.y; f.vr[3] = v23.z; f.vi[3] = v23.w;
    return f;
}

// acc += w * v for 4 polarisations: (wr + j wi)(vr + j vi) =
// wr vr - wi vi + j (wr vi + wi vr).  Records with w < 0 point into the
// conjugated copy of the bank, so no sign logic is needed here.
__device__ inline void fma_complex(float (&acc)[8], const float2 w, const RecVis &f) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        acc[2 * q] = fmaf(w.x, f.vr[q], fmaf(w.y, -f.vi[q], acc[2 * q]));
        acc[2 * q + 1] = fmaf(w.x, f.vi[q], fmaf(w.y, f.vr[q], acc[2 * q + 1]));
    }
}

__device__ inline void fma_real(float (&acc)[8], const float w, const RecVis &f) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        acc[2 * q] = fmaf(w, f.vr[q], acc[2 * q]);
        acc[2 * q + 1] = fmaf(w, f.vi[q], acc[2 * q + 1]);
    }
}

// Chunks are handed out through a per-launch counter (one vector atomic per
// chunk and workgroup), so workgroups that draw small chunks take more of
// them; chunk sizes vary from one record to R.  Each workgroup sees its
// chunks in increasing order.
__device__ inline uint32_t next_chunk(uint32_t *queue, uint32_t *slot) {
    __syncthreads();   // the previous value has been read by every wave
    if (threadIdx.x == 0) *slot = atomicAdd(queue, 1u);
    __syncthreads();
    return uniform_u32(*slot);
}

// ---------------------------------------------------------------------------
// moving-window gridder (supports up to 32)
// ---------------------------------------------------------------------------
// A footprint's S^2 cells are held by slots, slot (su, sv) owning the cells
// congruent to it mod S.  TEAM waves share one footprint, each holding a
// contiguous share of q = ceil(S^2 / TEAM) slots, at most KMAX per lane
// (q <= 64 KMAX); the workgroup's NW / TEAM teams take consecutive parts of
// each chunk's records, each team with its own window.
// Each slot keeps its cell and the term cell_v S + cell_u (W-projection;
// separable: cell_u and cell_v) of its tap offset (bytes, modulo 2^32); a
// record subtracts its own term, so the slot's tap offset costs one
// subtraction per record, and only slots whose cell leaves the footprint do
// more work.
// Work items are units: chunks of one tile over the planes of the launch's
// group.  An item's sums go to an LDS region covering what its chunks can
// touch, in fixed point, and from there to the grid once per item.
// Waves per workgroup: four single-wave teams, or eight waves in teams of
// TEAM (two such workgroups share a CU's LDS for supports up to 32, and the
// multi-wave instances are held to four waves per SIMD: beyond 128 VGPRs the
// eight-slot instance ran a third slower at three waves per SIMD).
constexpr int window_waves(int team) { return team == 1 ? 4 : 8; }
// Largest support of each window instance and its LDS region: 8 planes
// (polarisations x re/im) of int32, each plane kWindowTile + S - 1 cells
// square at most.  The plane stride is a compile-time constant, so the eight
// commits of a slot address one base with immediate offsets.
constexpr int kWindowTile = 16;
constexpr int window_smax(int kmax) { return kmax == 1 ? 8 : kmax == 4 ? 16 : 32; }
constexpr int window_plane(int kmax) {
    return (kWindowTile + window_smax(kmax) - 1) * (kWindowTile + window_smax(kmax) - 1);
}
// dynamic LDS of a window instance: the region and the unit slot
constexpr size_t window_lds(int kmax) { return sizeof(int32_t) * (8 * (size_t)window_plane(kmax) + 1); }

template <int KMAX, int TEAM, bool SEP, typename TapT>
__global__ __launch_bounds__(kWave * window_waves(TEAM))
__attribute__((amdgpu_waves_per_eu(TEAM > 1 ? 4 : 1))) void grid_window_kernel(
    const RecMeta *__restrict__ smeta, const float4 *__restrict__ svis, float *__restrict__ grid,
    const TapT *__restrict__ taps, const Chunk *__restrict__ chunks,
    const uint32_t *__restrict__ bucket_cfirst, const uint2 *__restrict__ units,
    const uint32_t *__restrict__ group_nunits, const PlaneLayout *__restrict__ planes,
    const int32_t *__restrict__ uinfo, uint32_t *__restrict__ queue, GridParams prm) {
    constexpr int NW = window_waves(TEAM);
    constexpr int NTEAMS = NW / TEAM;
    constexpr int PS = window_plane(KMAX);   // plane stride (cells)
    // [8][PS], plane q holding [RH][RW], then the workgroup's unit slot (the
    // region starts at LDS address 0, so commit addresses need no base)
    extern __shared__ int32_t region[];
    uint32_t *const s_next = reinterpret_cast<uint32_t *>(region + 8 * PS);
    constexpr uint32_t kElem = SEP ? sizeof(TapT) : 2 * sizeof(TapT);   // bytes per tap
    const int wave = (int)uniform_u32(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int team = wave / TEAM, member = wave % TEAM;
    const int npol = prm.npol;
    const char *tbase = reinterpret_cast<const char *>(taps);

    // the launch covers one plane group; its work items are the group's units
    const PlaneLayout gl = planes[prm.p_lo];
    const uint32_t ubase = bucket_cfirst[gl.base];
    const uint2 *gunits = units + ubase;
    const uint32_t nunits = group_nunits[prm.p_lo];
    for (uint32_t it = next_chunk(queue, s_next); it < nunits; it = next_chunk(queue, s_next)) {
        const uint2 un = gunits[it];
        const uint32_t c0 = un.x, c1 = un.x + un.y;
        // the item's region: union of its chunks' k_lo ranges (relative to
        // the tile origin) extended by their supports
        uint32_t umin = 0xffu, vmin = 0xffu, uend = 0u, vend = 0u;
        for (uint32_t c = c0; c < c1; ++c) {
            const Chunk ch = chunks[c];
            int pc;
            uint32_t tile_;
            bucket_plane_tile(gl, ch.bucket, &pc, &tile_);
            const uint32_t Sc = (uint32_t)planes[pc].S;
            umin = min(umin, ch.bbox & 0xffu);
            vmin = min(vmin, (ch.bbox >> 16) & 0xffu);
            uend = max(uend, ((ch.bbox >> 8) & 0xffu) + Sc);
            vend = max(vend, (ch.bbox >> 24) + Sc);
        }
        uint32_t tile;
        {
            int pc;
            bucket_plane_tile(gl, chunks[c0].bucket, &pc, &tile);
        }
        const uint32_t cu0 = ((tile % (uint32_t)gl.ntu) << gl.log2T) + umin;
        const uint32_t cv0 = ((tile / (uint32_t)gl.ntu) << gl.log2T) + vmin;
        const int RW = (int)(uend - umin);
        // byte offset in a region plane of cell (u, v): 4 (u - cu0) + 4 RW (v - cv0),
        // as one dot product of the packed cell with (4, 4 RW) plus a constant
        const uint32_t rstep = 4u | ((uint32_t)(4 * RW) << 16);
        const uint32_t rbias = 0u - 4u * (cu0 + (uint32_t)RW * cv0);
        const int RH = (int)(vend - vmin);
        const int plane_cells = RH * RW;

        // the unit's fixed-point exponent (its visibilities come scaled by
        // 2^scale); units with a non-finite visibility, or whose bound
        // overflows FP32, commit straight to the grid in FP32 (scale 0)
        const int32_t info = (int32_t)uniform_u32((uint32_t)uinfo[ubase + it]);
        const bool use_lds = (info & kUnitFixed) != 0;
        const int scale = unit_scale(info);
        if (use_lds) {
            for (int q = 0; q < 8; ++q)
                for (int i = threadIdx.x; i < plane_cells; i += NW * kWave) region[q * PS + i] = 0;
            __syncthreads();
        }
        // adds a slot's sums to its cell (fixed point: rounded to the nearest
        // quantum)
        auto commit = [&](float (&sums)[8], uint32_t cell_uv) {
            const uint32_t cu_ = cell_uv & 0xffffu, cv_ = cell_uv >> 16;
            if (use_lds) {
                // (the products are below 2^24 and the sum is the cell's
                // in-region offset, so the wrap of the bias cancels)
                int32_t *dst = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(region) +
                                                           dot_uv(cell_uv, rstep, rbias));
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    atomicAdd(&dst[q * PS], round_to_fixed(sums[q]));
            } else {
#pragma unroll
                for (int pol = 0; pol < 4; ++pol) {
                    if (pol < npol) {
                        float *dst = grid + 2 * (((int64_t)pol * prm.nv + cv_) * prm.nu + cu_);
                        unsafeAtomicAdd(dst, sums[2 * pol]);
                        unsafeAtomicAdd(dst + 1, sums[2 * pol + 1]);
                    }
                }
            }
        };

        for (uint32_t c = c0; c < c1; ++c) {
            const Chunk ch = chunks[c];
            int pc;
            uint32_t tile_;
            bucket_plane_tile(gl, ch.bucket, &pc, &tile_);
            const int S = planes[pc].S;
            // offset terms per cell step (bytes; phase-major table)
            const uint32_t su_step = kElem;
            const uint32_t sv_step = SEP ? kElem : (uint32_t)S * kElem;
            // the same steps packed (u, v) for the dot product with a cell
            const uint32_t uv_step = su_step | (sv_step << 16);

            // this wave's slots: member * q + k * 64 + lane (q = ceil(S^2 / TEAM));
            // per-lane flags are bit fields (bit k = slot k).  The slot count
            // per lane, KD = ceil(q / 64), is a compile-time constant of each
            // instance of the chunk's loop.
            const int nslots = S * S;
            const int q_ = (nslots + TEAM - 1) / TEAM;
            auto run = [&](auto kd_t) {
                constexpr int KD = decltype(kd_t)::value;
                uint32_t cell[KD], lo[KD], lov[KD], suv[KD];
                uint32_t valid_bits = 0;
                float acc[KD][8];
#pragma unroll
                for (int k = 0; k < KD; ++k) {
                    const int j = k * kWave + lane;
                    uint32_t sidx = (uint32_t)(member * q_ + j);
                    if (j < q_ && sidx < (uint32_t)nslots) valid_bits |= 1u << k;
                    // a spare lane mirrors a real slot: it follows the same
                    // cells and reads the same (in-bounds) taps, and its sums
                    // are never committed
                    else sidx %= (uint32_t)nslots;
                    // slot (su, sv) owns the cells congruent to it mod S
                    const uint32_t sv = sidx / (uint32_t)S;
                    suv[k] = (sidx - sv * (uint32_t)S) | (sv << 16);
                    cell[k] = kNoCell;
                    lo[k] = 0u;
                    lov[k] = 0u;
#pragma unroll
                    for (int q = 0; q < 8; ++q) acc[k][q] = 0.0f;
                }

                // window of the current footprint: slots whose cell left it commit
                // and take the cell congruent to them inside the new footprint
                uint32_t prev_kuv = 0xffffffffu;
                uint32_t ru = 0, rv = 0;   // the record's offset terms (bytes, modulo 2^32)
                auto window_update = [&](const RecMeta m) {
                    const uint32_t kuv = m.kuv;
                    if (kuv == prev_kuv) return;
                    prev_kuv = kuv;
                    const uint32_t ku = meta_ku(m), kv = meta_kv(m);
                    const uint32_t kmu = ku % (uint32_t)S, kmv = kv % (uint32_t)S;
                    // (u, v) pairs in 16-bit halves: the footprint origin, its
                    // residues mod S and S itself
                    const u16x2 korg = as_u16x2(kuv), kres = as_u16x2(kmu | (kmv << 16)),
                                ss = as_u16x2((uint32_t)S | ((uint32_t)S << 16));
#pragma unroll
                    for (int k = 0; k < KD; ++k) {
                        // the slot's cell has left the footprint (a borrow
                        // only where du < 0); the test runs on the exec mask
                        const uint32_t d = cell[k] - kuv;
                        if (max(d & 0xffffu, d >> 16) >= (uint32_t)S) {
                            if (((valid_bits >> k) & 1u) && cell[k] != kNoCell)
                                commit(acc[k], cell[k]);
#pragma unroll
                            for (int q = 0; q < 8; ++q) acc[k][q] = 0.0f;
                            // the cell congruent to the slot in the footprint:
                            // origin + (slot - origin mod S) mod S, per half; a
                            // negative difference wraps above 2^15, and adding S
                            // brings it back below S, so the smaller of the two
                            // is the residue
                            const u16x2 dd = as_u16x2(suv[k]) - kres;
                            const u16x2 cc = korg + __builtin_elementwise_min(dd, dd + ss);
                            cell[k] = as_u32(cc);
                            // cells < 2^16 and steps < 2^10: the products
                            // and their sum are exact
                            if constexpr (SEP) {
                                lo[k] = dot_uv(cell[k], su_step, 0u);
                                lov[k] = dot_uv(cell[k], sv_step << 16, 0u);
                            } else {
                                lo[k] = dot_uv(cell[k], uv_step, 0u);
                            }
                        }
                    }
                    if constexpr (SEP) {
                        ru = ku * su_step;
                        rv = kv * sv_step;
                    } else {
                        ru = kv * sv_step + ku * su_step;
                    }
                };

                // tap of slot k for a record (uniform base + 32-bit lane offset)
                auto tap = [&](const RecMeta m, const int k) {
                    if constexpr (SEP) {
                        const char *tu = tbase + (size_t)(m.toff & 0xffffu) * kElem;
                        const char *tv = tbase + (size_t)(m.toff >> 16) * kElem;
                        const uint32_t ou = lo[k] - ru, ov = lov[k] - rv;
                        return make_float2(TapTraits<TapT>::real((const TapT *)(tu + ou), 0) *
                                               TapTraits<TapT>::real((const TapT *)(tv + ov), 0),
                                           0.0f);
                    } else {
                        const char *tb = tbase + (size_t)m.toff * kElem;
                        uint32_t o = lo[k] - ru;
                        asm volatile("" : "+v"(o));   // keeps the offset 32-bit: scalar-base load
                        return TapTraits<TapT>::cplx((const TapT *)(tb + o), 0);
                    }
                };
                auto madd = [&](const int k, const float2 w, const RecVis &f) {
                    if constexpr (SEP)
                        fma_real(acc[k], w.x, f);
                    else
                        fma_complex(acc[k], w, f);
                };

                const uint32_t len = ch.len;
                const uint32_t rb = ch.start + (uint32_t)(((uint64_t)len * team) / NTEAMS);
                const uint32_t re = ch.start + (uint32_t)(((uint64_t)len * (team + 1)) / NTEAMS);
                if (rb < re) {
                    // records are read in batches on the scalar unit; the next
                    // batch's loads are issued after the current batch has been
                    // consumed (scalar loads complete out of order: waiting for
                    // one is waiting for all), so they overlap the current
                    // batch's multiply-adds
                    RecMeta nm[kBatch];
                    float4 na4[kBatch], nb4[kBatch];
                    // the record arrays are padded (kRecPad entries), so a batch
                    // may run past the chunk's end (those records are not used)
                    const RecMeta *pm = smeta + rb;
                    const float4 *pv = svis + 2 * (size_t)rb;
                    auto load_batch = [&]() {
#pragma unroll
                        for (int i = 0; i < kBatch; ++i) {
                            nm[i] = pm[i];
                            na4[i] = pv[2 * i];
                            nb4[i] = pv[2 * i + 1];
                        }
                        pm += kBatch;
                        pv += 2 * kBatch;
                    };
                    load_batch();
                    wait_scalar_loads();
                    for (uint32_t r = rb; r < re; r += kBatch) {
                        RecMeta mm[kBatch];
                        float4 va4[kBatch], vb4[kBatch];
#pragma unroll
                        for (int i = 0; i < kBatch; ++i) {
                            mm[i] = nm[i];
                            va4[i] = na4[i];
                            vb4[i] = nb4[i];
                        }
                        __builtin_amdgcn_sched_barrier(0);
                        load_batch();
#pragma unroll
                        for (int i = 0; i < kBatch; ++i) {
                            if (r + (uint32_t)i < re) {
                                window_update(mm[i]);
                                const RecVis f = unpack_vis(va4[i], vb4[i]);
                                float2 w[KD];
#pragma unroll
                                for (int k = 0; k < KD; ++k)
                                    w[k] = tap(mm[i], k);
#pragma unroll
                                for (int k = 0; k < KD; ++k)
                                    madd(k, w[k], f);
                            }
                        }
                    }
#pragma unroll
                    for (int k = 0; k < KD; ++k)
                        if (((valid_bits >> k) & 1u) && cell[k] != kNoCell)
                            commit(acc[k], cell[k]);
                }
            };
            const int kdyn = (q_ + kWave - 1) / kWave;
            if constexpr (KMAX == 1) {
                run(std::integral_constant<int, 1>{});
            } else if constexpr (KMAX == 4) {
                switch (kdyn) {
                case 1: run(std::integral_constant<int, 1>{}); break;
                case 2: run(std::integral_constant<int, 2>{}); break;
                case 3: run(std::integral_constant<int, 3>{}); break;
                default: run(std::integral_constant<int, 4>{}); break;
                }
            } else {
                static_assert(KMAX == 8, "slot counts 1..8");
                switch (kdyn) {
                case 1: run(std::integral_constant<int, 1>{}); break;
                case 2: run(std::integral_constant<int, 2>{}); break;
                case 3: run(std::integral_constant<int, 3>{}); break;
                case 4: run(std::integral_constant<int, 4>{}); break;
                case 5: run(std::integral_constant<int, 5>{}); break;
                case 6: run(std::integral_constant<int, 6>{}); break;
                case 7: run(std::integral_constant<int, 7>{}); break;
                default: run(std::integral_constant<int, 8>{}); break;
                }
            }
        }

        if (use_lds) {
            __syncthreads();
            // cell j = rv * RW + ru of each polarisation's plane; a thread
            // steps j by the workgroup size, so its (rv, ru) advance by a
            // fixed step (no division per cell)
            constexpr int kThreads = NW * kWave;
            const int step_u = kThreads % RW, step_v = kThreads / RW;
            const int ru0 = (int)threadIdx.x % RW, rv0 = (int)threadIdx.x / RW;
            for (int pol = 0; pol < npol; ++pol) {
                const int32_t *qre = region + (2 * pol) * PS;
                const int32_t *qim = qre + PS;
                float *gp = grid + 2 * (((int64_t)pol * prm.nv + cv0) * prm.nu + cu0);
                int ru_ = ru0, rv_ = rv0;
                for (int j = threadIdx.x; j < plane_cells; j += kThreads) {
                    const int32_t qr = qre[j], qi = qim[j];
                    if ((qr | qi) != 0) {
                        float *dst = gp + 2 * ((int64_t)rv_ * prm.nu + ru_);
                        unsafeAtomicAdd(dst, ldexpf((float)qr, -scale));
                        unsafeAtomicAdd(dst + 1, ldexpf((float)qi, -scale));
                    }
                    ru_ += step_u;
                    rv_ += step_v;
                    if (ru_ >= RW) {
                        ru_ -= RW;
                        ++rv_;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// blocked output-stationary gridder (large supports)
// ---------------------------------------------------------------------------
// The grid region a unit can touch (its tile plus the group's largest S - 1
// halo) is cut into 8 x 8-cell blocks, one cell per lane; block b belongs to
// wave b mod NW of the workgroup (its k-th block is b = k NW + wave), and its
// 8 accumulators per lane stay in registers for the whole unit.  Every wave
// walks all records of the unit (scalar loads).  Per record, lane k of a
// wave tests block k against the record's footprint, so one vector compare
// and a ballot give the wave's overlapped blocks (and those lying wholly
// inside the footprint, which need no per-lane mask); each overlapped block
// then takes one tap load and 16 multiply-adds per lane.  Nothing is
// committed until the unit ends; then each touched cell is added to the
// grid with float atomics.  Where records are sparse, as in the high-|w|
// planes of large support, this replaces the moving window's per-record
// slot commits; the lane utilisation is S^2 over the overlapped blocks'
// cells, about (S/(S+7))^2.
// W-projection instances are held to 128 VGPRs (four waves per SIMD), which
// they fit without spilling; separable ones need a few more registers.
template <int KMAX, int NW, bool SEP, typename TapT>
__global__ __launch_bounds__(NW * kWave) __attribute__((amdgpu_waves_per_eu(SEP ? 1 : 4)))
void grid_block_kernel(
    const RecMeta *__restrict__ smeta, const float4 *__restrict__ svis, float *__restrict__ grid,
    const TapT *__restrict__ taps, const Chunk *__restrict__ chunks,
    const uint32_t *__restrict__ bucket_cfirst, const uint2 *__restrict__ units,
    const uint32_t *__restrict__ group_nunits, const PlaneLayout *__restrict__ planes,
    const int32_t *__restrict__ uinfo, uint32_t *__restrict__ queue, GridParams prm) {
    // Lanes outside a footprint normally multiply a zero tap, which adds
    // nothing; a non-finite visibility would turn that into NaN, so units
    // holding one take the masked path instead.
    constexpr uint32_t kElem = SEP ? sizeof(TapT) : 2 * sizeof(TapT);   // bytes per tap
    const int wave = (int)uniform_u32(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int lu = lane & 7, lv = lane >> 3;
    const int npol = prm.npol;
    const char *tbase = reinterpret_cast<const char *>(taps);

    // The launch covers one plane group.  Its work comes in units: chunks of
    // one tile (in any of the group's planes), accumulated together in
    // registers and committed once per unit over the tile's region (the
    // tile plus the group's largest halo).
    const PlaneLayout g0 = planes[prm.p_lo];
    const int Tm = g0.T - 1;
    const uint32_t ntu = (uint32_t)g0.ntu;
    const uint32_t gn = (uint32_t)g0.grp_n;
    const uint32_t gbase = (uint32_t)g0.base;
    const uint32_t nunits = group_nunits[prm.p_lo];
    const uint2 *gunits = units + bucket_cfirst[gbase];
    const int nbx = (g0.T + g0.grp_smax - 1 + 7) >> 3;
    const int nblocks = nbx * nbx;

    // lane k < KMAX: origin of the wave's block k, for the overlap tests
    uint32_t blo_u = 0xffff0000u, blo_v = 0xffff0000u;   // never overlaps
    {
        const int b = lane * NW + wave;
        if (lane < KMAX && b < nblocks) {
            blo_u = (uint32_t)((b % nbx) << 3);
            blo_v = (uint32_t)((b / nbx) << 3);
        }
    }
    // per block: this lane's cell (packed u | v << 16, region-relative)
    uint32_t cuv[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int b = k * NW + wave;
        cuv[k] = (uint32_t)(((b % nbx) << 3) + lu) | ((uint32_t)(((b / nbx) << 3) + lv) << 16);
    }

    __shared__ uint32_t s_next;
    const uint32_t ubase = bucket_cfirst[gbase];
    // the exact or fast path is chosen per unit
    for (uint32_t i = next_chunk(queue, &s_next); i < nunits; i = next_chunk(queue, &s_next)) {
        const bool exact_unit =
            (uniform_u32((uint32_t)uinfo[ubase + i]) & (uint32_t)kUnitNonFinite) != 0u;
        auto work = [&](auto exact_t) {
            const uint2 un = gunits[i];
            const uint32_t c0 = un.x, c1 = un.x + un.y;
            const uint32_t t = (chunks[c0].bucket - gbase) / gn;
            const int cu0 = (int)((t % ntu) << g0.log2T);
            const int cv0 = (int)((t / ntu) << g0.log2T);

            float acc[KMAX][8];
#pragma unroll
            for (int k = 0; k < KMAX; ++k)
#pragma unroll
                for (int q = 0; q < 8; ++q) acc[k][q] = 0.0f;
            uint32_t touched = 0;

            for (uint32_t c = c0; c < c1; ++c) {
                const Chunk ch = chunks[c];
                const int p = g0.grp_first + (int)((ch.bucket - gbase) % gn);
                const PlaneLayout pl = planes[p];
                const int S = pl.S;
                // this lane's tap offset in each block, in bytes relative to
                // the footprint's first tap
                uint32_t voff[KMAX], voffv[KMAX];
#pragma unroll
                for (int k = 0; k < KMAX; ++k) {
                    const uint32_t cu = cuv[k] & 0xffffu, cv = cuv[k] >> 16;
                    if constexpr (SEP) {
                        voff[k] = cu * kElem;
                        voffv[k] = cv * kElem;
                    } else {
                        voff[k] = (cv * (uint32_t)S + cu) * kElem;
                        voffv[k] = 0u;
                    }
                }

                auto visit = [&](const RecMeta m, const RecVis &f, auto exact_t) {
                    constexpr bool EXACT = decltype(exact_t)::value;
                    // footprint origin relative to the region
                    const uint32_t a = meta_ku(m) & (uint32_t)Tm;
                    const uint32_t bq = meta_kv(m) & (uint32_t)Tm;
                    // block [lo, lo+7] overlaps [a, a+S-1] iff lo + 7 - a in
                    // [0, S+6]; it lies inside iff lo - a in [0, S-8]
                    const uint32_t hit = (uint32_t)__ballot((blo_u + 7u - a <= (uint32_t)(S + 6)) &&
                                                            (blo_v + 7u - bq <= (uint32_t)(S + 6)));
                    const uint32_t full = (uint32_t)__ballot((blo_u - a <= (uint32_t)(S - 8)) &&
                                                             (blo_v - bq <= (uint32_t)(S - 8)));
                    touched |= hit;
                    const uint32_t ab = a | (bq << 16);
                    const char *tb_;
                    const char *tbv = nullptr;
                    if constexpr (SEP) {
                        tb_ = tbase + ((int64_t)(m.toff & 0xffffu) - (int64_t)a) * (int64_t)kElem;
                        tbv = tbase + ((int64_t)(m.toff >> 16) - (int64_t)bq) * (int64_t)kElem;
                    } else {
                        tb_ = tbase + ((int64_t)m.toff - (int64_t)(bq * (uint32_t)S + a)) * (int64_t)kElem;
                    }
                    // tap of lane's cell in block k (uniform base + 32-bit lane offset)
                    auto tap = [&](const int k) {
                        uint32_t o = voff[k];
                        asm volatile("" : "+v"(o));   // keeps the offset 32-bit: scalar-base load
                        if constexpr (SEP) {
                            uint32_t ov = voffv[k];
                            asm volatile("" : "+v"(ov));
                            const float t_ = TapTraits<TapT>::real((const TapT *)(tb_ + o), 0) *
                                             TapTraits<TapT>::real((const TapT *)(tbv + ov), 0);
                            return make_float2(t_, 0.0f);
                        } else {
                            return TapTraits<TapT>::cplx((const TapT *)(tb_ + o), 0);
                        }
                    };
                    auto madd = [&](const int k, const float2 w) {
                        if constexpr (SEP)
                            fma_real(acc[k], w.x, f);
                        else
                            fma_complex(acc[k], w, f);
                    };
                    if constexpr (EXACT) {
#pragma unroll
                        for (int k = 0; k < KMAX; ++k) {
                            if (!((hit >> k) & 1u)) continue;
                            const uint32_t d = cuv[k] - ab;   // a borrow only where du < 0
                            if (((full >> k) & 1u) || max(d & 0xffffu, d >> 16) < (uint32_t)S)
                                madd(k, tap(k));
                        }
                    } else {
                        // all tap loads of the record first, then the
                        // multiply-adds; lanes outside the footprint keep a
                        // zero tap (one vector test per overlapped block)
                        float2 w[KMAX];
#pragma unroll
                        for (int k = 0; k < KMAX; ++k) {
                            w[k] = make_float2(0.0f, 0.0f);
                            if (!((hit >> k) & 1u)) continue;
                            const uint32_t d = cuv[k] - ab;
                            if (max(d & 0xffffu, d >> 16) < (uint32_t)S) w[k] = tap(k);
                        }
#pragma unroll
                        for (int k = 0; k < KMAX; ++k)
                            if ((hit >> k) & 1u) madd(k, w[k]);
                    }
                };

                auto records = [&](auto exact_t) {
                    const uint32_t rb = ch.start, re = ch.start + ch.len;
                    RecMeta nm[kBatch];
                    float4 na4[kBatch], nb4[kBatch];
                    // the record arrays are padded (kRecPad entries), so a
                    // batch may run past the chunk's end (those are not used)
                    const RecMeta *pm = smeta + rb;
                    const float4 *pv = svis + 2 * (size_t)rb;
                    auto load_batch = [&]() {
#pragma unroll
                        for (int i = 0; i < kBatch; ++i) {
                            nm[i] = pm[i];
                            na4[i] = pv[2 * i];
                            nb4[i] = pv[2 * i + 1];
                        }
                        pm += kBatch;
                        pv += 2 * kBatch;
                    };
                    load_batch();
                    wait_scalar_loads();
                    for (uint32_t r = rb; r < re; r += kBatch) {
                        RecMeta mm[kBatch];
                        float4 va4[kBatch], vb4[kBatch];
#pragma unroll
                        for (int i = 0; i < kBatch; ++i) {
                            mm[i] = nm[i];
                            va4[i] = na4[i];
                            vb4[i] = nb4[i];
                        }
                        __builtin_amdgcn_sched_barrier(0);
                        load_batch();
#pragma unroll
                        for (int i = 0; i < kBatch; ++i)
                            if (r + (uint32_t)i < re) visit(mm[i], unpack_vis(va4[i], vb4[i]), exact_t);
                    }
                };
                records(exact_t);
            }

            // commit: one float atomic per touched cell, polarisation and part
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                if (!((touched >> k) & 1u)) continue;
                const int u = cu0 + (int)(cuv[k] & 0xffffu), v = cv0 + (int)(cuv[k] >> 16);
                if (u >= prm.nu || v >= prm.nv) continue;
#pragma unroll
                for (int pol = 0; pol < 4; ++pol) {
                    if (pol < npol && (acc[k][2 * pol] != 0.0f || acc[k][2 * pol + 1] != 0.0f)) {
                        float *dst = grid + 2 * (((int64_t)pol * prm.nv + v) * prm.nu + u);
                        unsafeAtomicAdd(dst, acc[k][2 * pol]);
                        unsafeAtomicAdd(dst + 1, acc[k][2 * pol + 1]);
                    }
                }
            }
        };
        if (exact_unit)
            work(std::true_type{});
        else
            work(std::false_type{});
    }
}

// Gathers the visibilities of one plane group's units into sorted order,
// padded to 4 polarisations, and writes each unit's word (see kUnitFixed).
// A workgroup takes a unit (at most kGatherThreads * kGatherPerThread
// records, contiguous in sorted order): every thread first loads the
// permutation entries of its records, then their visibilities (all loads in
// flight together), bounds the unit's partial sums, and for the window
// classes (fixed = 1) stores the visibilities multiplied by the unit's
// power-of-two scale.
constexpr int kGatherThreads = 256;
constexpr int kGatherPerThread = 8;   // R <= 2048 records per unit

__global__ __launch_bounds__(kGatherThreads) void gather_units_kernel(
    const PlaneLayout *__restrict__ planes, int32_t g, int32_t sep, int32_t fixed,
    const uint32_t *__restrict__ bucket_cfirst, const uint2 *__restrict__ units,
    const uint32_t *__restrict__ group_nunits, const Chunk *__restrict__ chunks,
    const uint32_t *__restrict__ sperm, const float2 *__restrict__ vis, int32_t npol,
    float4 *__restrict__ svis, int32_t *__restrict__ uinfo) {
    __shared__ float s_part[kGatherThreads / kWave];
    __shared__ int s_bad[kGatherThreads / kWave];
    const PlaneLayout gl = planes[g];
    const uint32_t ubase = bucket_cfirst[gl.base];
    const uint32_t n = group_nunits[g];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (uint32_t it = blockIdx.x; it < n; it += gridDim.x) {
        const uint2 un = units[ubase + it];
        const uint32_t c0 = un.x, c1 = un.x + un.y;
        const uint32_t rs = chunks[c0].start;
        const Chunk last = chunks[c1 - 1];
        const uint32_t re = last.start + last.len;
        uint32_t idx[kGatherPerThread];
#pragma unroll
        for (int k = 0; k < kGatherPerThread; ++k) {
            const uint32_t r = rs + threadIdx.x + (uint32_t)k * kGatherThreads;
            idx[k] = (r < re) ? sperm[r] : 0u;
        }
        float4 a[kGatherPerThread], b[kGatherPerThread];
#pragma unroll
        for (int k = 0; k < kGatherPerThread; ++k) {
            const uint32_t r = rs + threadIdx.x + (uint32_t)k * kGatherThreads;
            a[k] = b[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (r >= re) continue;
            const float2 *v = vis + (size_t)idx[k] * npol;
            if (npol == 4) {
                a[k] = reinterpret_cast<const float4 *>(v)[0];
                b[k] = reinterpret_cast<const float4 *>(v)[1];
            } else {
                float2 x[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) x[q] = (q < npol) ? v[q] : make_float2(0.0f, 0.0f);
                a[k] = make_float4(x[0].x, x[0].y, x[1].x, x[1].y);
                b[k] = make_float4(x[2].x, x[2].y, x[3].x, x[3].y);
            }
        }
        // bound: sum over the records of the plane's largest weight component
        // times the record's largest visibility component (the chunk of a
        // record, hence its plane, only moves forward with r)
        float part = 0.0f;
        bool bad = false;
        uint32_t c = c0;
        uint32_t cend = chunks[c0].start + chunks[c0].len;
        float wmax = 0.0f;
        {
            int pc;
            uint32_t tile_;
            bucket_plane_tile(gl, chunks[c0].bucket, &pc, &tile_);
            const float t = planes[pc].tmax;
            wmax = sep ? t * t : t;
        }
#pragma unroll
        for (int k = 0; k < kGatherPerThread; ++k) {
            const uint32_t r = rs + threadIdx.x + (uint32_t)k * kGatherThreads;
            if (r >= re) continue;
            while (r >= cend) {
                ++c;
                const Chunk ch = chunks[c];
                cend = ch.start + ch.len;
                int pc;
                uint32_t tile_;
                bucket_plane_tile(gl, ch.bucket, &pc, &tile_);
                const float t = planes[pc].tmax;
                wmax = sep ? t * t : t;
            }
            const float m = fmaxf(fmaxf(fmaxf(fabsf(a[k].x), fabsf(a[k].y)), fmaxf(fabsf(a[k].z), fabsf(a[k].w))),
                                  fmaxf(fmaxf(fabsf(b[k].x), fabsf(b[k].y)), fmaxf(fabsf(b[k].z), fabsf(b[k].w))));
            part += wmax * m;
            bad = bad || !(isfinite(a[k].x) && isfinite(a[k].y) && isfinite(a[k].z) &&
                           isfinite(a[k].w) && isfinite(b[k].x) && isfinite(b[k].y) &&
                           isfinite(b[k].z) && isfinite(b[k].w));
        }
        for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
        const bool wbad = __any(bad);
        if (lane == 0) {
            s_part[wave] = part;
            s_bad[wave] = wbad ? 1 : 0;
        }
        __syncthreads();
        float bound = 0.0f;
        int anybad = 0;
        for (int w = 0; w < kGatherThreads / kWave; ++w) {
            bound += s_part[w];
            anybad |= s_bad[w];
        }
        __syncthreads();   // s_part is rewritten by the next unit
        // margin for the rounding of the sums above
        bound = 2.0f * bound * 1.0001f + 1e-30f;
        int scale = 0;
        int32_t info = anybad ? kUnitNonFinite : 0;
        if (fixed && !anybad && isfinite(bound)) {
            int e = 0;
            frexpf(bound, &e);   // bound < 2^e
            scale = max(-120, min(120, 30 - e));
            info |= kUnitFixed;
        }
        info |= (scale + 128) & 0xff;
        if (threadIdx.x == 0) uinfo[ubase + it] = info;
        const float fs = ldexpf(1.0f, scale);
#pragma unroll
        for (int k = 0; k < kGatherPerThread; ++k) {
            const uint32_t r = rs + threadIdx.x + (uint32_t)k * kGatherThreads;
            if (r >= re) continue;
            float4 x = a[k], y = b[k];
            if (scale != 0) {
                x.x *= fs; x.y *= fs; x.z *= fs; x.w *= fs;
                y.x *= fs; y.y *= fs; y.z *= fs; y.w *= fs;
            }
            svis[2 * (size_t)r] = x;
            svis[2 * (size_t)r + 1] = y;
        }
    }
}

__global__ void clear_words_kernel(uint32_t *w, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) w[i] = 0u;
}

struct GridPtrs {
    const RecMeta *smeta;
    const float4 *svis;
    float *grid;
    const void *taps;
    const Chunk *chunks;
    const uint32_t *bucket_cfirst;
    const uint2 *units;
    const uint32_t *group_nunits;
    const PlaneLayout *planes;
    const int32_t *uinfo;        // per-unit words written by the gather
    uint32_t *queue;             // this launch's unit counter
};

template <int KMAX, int TEAM, bool SEP, typename TapT>
void launch_window(const GridPtrs &a, const GridParams &prm, size_t lds, hipStream_t stream) {
    auto kern = grid_window_kernel<KMAX, TEAM, SEP, TapT>;
    const int threads = kWave * window_waves(TEAM);
    hipLaunchKernelGGL(kern, dim3(resident_groups((const void *)kern, threads, lds)),
                       dim3(threads), lds, stream, a.smeta, a.svis, a.grid, (const TapT *)a.taps,
                       a.chunks, a.bucket_cfirst, a.units, a.group_nunits, a.planes, a.uinfo,
                       a.queue, prm);
}

template <int KMAX, int NW, bool SEP, typename TapT>
void launch_block(const GridPtrs &a, const GridParams &prm, hipStream_t stream) {
    auto kern = grid_block_kernel<KMAX, NW, SEP, TapT>;
    hipLaunchKernelGGL(kern, dim3(resident_groups((const void *)kern, NW * kWave, 0)),
                       dim3(NW * kWave), 0, stream, a.smeta, a.svis, a.grid, (const TapT *)a.taps,
                       a.chunks, a.bucket_cfirst, a.units, a.group_nunits, a.planes, a.uinfo,
                       a.queue, prm);
}

// Largest region, in 8 x 8 blocks, of a chunk of tile side T and support S.
inline int region_blocks(int T, int S) {
    const int side = (T + S - 1 + 7) / 8;
    return side * side;
}

template <bool SEP, typename TapT>
hipError_t launch_class(int cls, const GridPtrs &a, const GridParams &prm, int smax, int tile,
                        hipStream_t stream) {
    // LDS region of the window gridders: 8 planes of the instance's fixed
    // stride (tile plus the class's largest halo)
    if (cls <= 2 && (tile != kWindowTile || smax > window_smax(cls == 0 ? 1 : cls == 1 ? 4 : 8)))
        return hipErrorInvalidValue;
    switch (cls) {
    case 0: launch_window<1, 1, SEP, TapT>(a, prm, window_lds(1), stream); break;
    case 1: launch_window<4, 1, SEP, TapT>(a, prm, window_lds(4), stream); break;
    case 2: launch_window<8, 2, SEP, TapT>(a, prm, window_lds(8), stream); break;
    default:
        if (region_blocks(tile, smax) > 7 * 16) return hipErrorInvalidValue;
        launch_block<7, 16, SEP, TapT>(a, prm, stream);
        break;
    }
    return hipGetLastError();
}

template <bool SEP>
hipError_t launch_class_t(mg_dtype dt, int cls, const GridPtrs &a, const GridParams &prm,
                          int smax, int tile, hipStream_t stream) {
    switch (dt) {
    case MG_F16: return launch_class<SEP, __half>(cls, a, prm, smax, tile, stream);
    case MG_BF16: return launch_class<SEP, __hip_bfloat16>(cls, a, prm, smax, tile, stream);
    default: return launch_class<SEP, float>(cls, a, prm, smax, tile, stream);
    }
}

}  // namespace

namespace {
template <typename F>
size_t walk_grid_scratch(const PlanState &P, F &&place) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += arena_round(bytes);
        return at;
    };
    place(0, take(sizeof(float4) * 2 * (size_t)(P.nrec + kRecPad)));
    place(1, take(sizeof(int32_t) * (size_t)P.max_chunks));
    place(2, take(sizeof(uint32_t) * (size_t)P.nplanes_eff));
    return off;
}
}  // namespace

size_t grid_scratch_bytes(const PlanState &P) {
    return walk_grid_scratch(P, [](int, size_t) {});
}

mg_status launch_grid(const PlanState &P, const void *vis, void *grid, void *scratch,
                      hipStream_t stream) {
    if (P.nrec == 0) return MG_OK;
    hipError_t e = hipSuccess;
    void *own = nullptr;
    if (!scratch) {
        e = scratch_alloc(&own, grid_scratch_bytes(P), stream);
        if (e != hipSuccess) return set_error(MG_ENOMEM, "grid: scratch allocation failed");
        scratch = own;
    }
    GridScratch gs;
    walk_grid_scratch(P, [&](int what, size_t at) {
        void *p = static_cast<char *>(scratch) + at;
        if (what == 0) gs.svis = static_cast<float4 *>(p);
        else if (what == 1) gs.uinfo = static_cast<int32_t *>(p);
        else gs.queues = static_cast<uint32_t *>(p);
    });
    const int np = P.nplanes_eff;
    const bool sep = P.kind == MG_KERNEL_SEPARABLE;
    hipLaunchKernelGGL(clear_words_kernel, dim3(1), dim3(256), 0, stream, gs.queues, np);
    // sorted, scaled visibilities and unit words, one launch per plane group
    const int gather_groups = resident_groups((const void *)gather_units_kernel, kGatherThreads, 0);
    for (int p = 0; p < np; p += P.planes[p].grp_n)
        hipLaunchKernelGGL(gather_units_kernel, dim3(gather_groups), dim3(kGatherThreads), 0,
                           stream, P.d_planes, p, (int32_t)sep,
                           (int32_t)(P.planes[p].cls <= 2), P.bucket_cfirst, P.units,
                           P.group_nunits, P.chunks, P.sperm, (const float2 *)vis, P.geom.npol,
                           gs.svis, gs.uinfo);
    GridPtrs a{P.smeta,   gs.svis,        (float *)grid, P.taps,   P.chunks, P.bucket_cfirst,
               P.units,   P.group_nunits, P.d_planes,   gs.uinfo, nullptr};
    GridParams prm{P.geom.npol, P.geom.nu, P.geom.nv, P.geom.beta, 0, 0};
    // one launch per run of consecutive planes of the same class
    int p0 = 0;
    while (p0 < np && e == hipSuccess) {
        int p1 = p0 + 1;
        int smax = P.planes[p0].S;
        while (p1 < np && P.planes[p1].cls == P.planes[p0].cls) {
            smax = std::max(smax, P.planes[p1].S);
            ++p1;
        }
        prm.p_lo = p0;
        prm.p_hi = p1;
        const int cls = P.planes[p0].cls;
        a.queue = gs.queues + p0;
        e = sep ? launch_class_t<true>(P.tap_dtype, cls, a, prm, smax, P.planes[p0].T, stream)
                : launch_class_t<false>(P.tap_dtype, cls, a, prm, smax, P.planes[p0].T, stream);
        p0 = p1;
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (own) scratch_free(own, stream);
    if (e != hipSuccess) return set_error(MG_EDEVICE, std::string("grid kernels: ") + hipGetErrorString(e));
    return MG_OK;
}

}  // namespace mg
