// Plan building: index rule, bucket counting sort, chunk list, per-chunk
// cell sort.
//
// The thesis sorts records by their position on the virtual NN grid before
// gridding ("SS" ordering, Section 3.2.4) because the order in which records
// reach the gridder sets how often accumulated values have to be committed
// (Chapter 4).  Here the order is (plane, uv tile, cell): a counting sort by
// (plane, tile) bucket over the whole record set, then a counting sort by
// cell inside each chunk of at most R records.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace mg {

namespace {

constexpr uint32_t kInvalidBucket = 0xffffffffu;

// ---------------------------------------------------------------------------
// index rule -> bucket histogram and skipped count; the scatter evaluates the
// rule again (reading uvw costs what storing and re-reading its results
// would, and saves writing them)
// ---------------------------------------------------------------------------
// Packed meta and bucket of record r (bucket kInvalidBucket if skipped).
template <typename T>
__device__ inline RecIndex index_bucket(const DevGeom &g, const PlaneLayout *planes,
                                        const T *uvw, int64_t r, uint32_t *bucket) {
    const RecIndex ix = index_record<T>(g, uvw[3 * r], uvw[3 * r + 1], uvw[3 * r + 2]);
    uint32_t b = kInvalidBucket;
    if (ix.valid) {
        const int p = ix.plane < 0 ? 0 : ix.plane;
        const PlaneLayout pl = planes[p];
        const uint32_t tu = (uint32_t)ix.ku >> pl.log2T;
        const uint32_t tv = (uint32_t)ix.kv >> pl.log2T;
        b = (uint32_t)(pl.base + ((int64_t)tv * pl.ntu + tu) * pl.grp_n + (p - pl.grp_first));
    }
    *bucket = b;
    return ix;
}

template <typename T>
__global__ __launch_bounds__(256) void index_bucket_kernel(
    DevGeom g, const PlaneLayout *__restrict__ planes, int64_t nrec, const T *__restrict__ uvw,
    uint32_t *__restrict__ hist, int64_t *__restrict__ counters) {
    __shared__ uint32_t s_skip;
    if (threadIdx.x == 0) s_skip = 0;
    __syncthreads();
    uint32_t skipped = 0;
    // every lane of a wave runs the same number of iterations (the
    // aggregated atomic needs the whole wave)
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
    for (int64_t r0 = first; r0 < nrec; r0 += stride) {
        const int64_t r = r0 + (threadIdx.x & 63);
        const bool in = r < nrec;
        uint32_t b = kInvalidBucket;
        if (in) index_bucket<T>(g, planes, uvw, r, &b);
        if (in && b == kInvalidBucket) ++skipped;
        wave_counter_add(hist, b, b != kInvalidBucket, false);
    }
    if (skipped) atomicAdd(&s_skip, skipped);
    __syncthreads();
    if (threadIdx.x == 0 && s_skip) atomicAdd((unsigned long long *)&counters[0],
                                              (unsigned long long)s_skip);
}

// ---------------------------------------------------------------------------
// exclusive scan of (count, chunks-of-R) pairs over the buckets
// ---------------------------------------------------------------------------
constexpr int kScanItems = 16;
constexpr int kScanBlock = 256 * kScanItems;

__device__ inline uint2 pair_of(const uint32_t *hist, int64_t i, int64_t n, uint32_t R) {
    if (i >= n) return make_uint2(0, 0);
    uint32_t c = hist[i];
    return make_uint2(c, (c + R - 1) / R);
}

__device__ inline uint2 add2(uint2 a, uint2 b) { return make_uint2(a.x + b.x, a.y + b.y); }

// Block-wide exclusive scan of one uint2 per thread (256 threads).
__device__ inline uint2 block_exclusive_scan(uint2 v, uint2 *total) {
    __shared__ uint2 s[256];
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint2 add = (t >= off) ? s[t - off] : make_uint2(0, 0);
        __syncthreads();
        s[t] = add2(s[t], add);
        __syncthreads();
    }
    uint2 incl = s[t];
    *total = s[255];
    __syncthreads();
    return make_uint2(incl.x - v.x, incl.y - v.y);
}

__global__ __launch_bounds__(256) void scan_reduce_kernel(const uint32_t *__restrict__ hist,
                                                          int64_t n, uint32_t R,
                                                          uint2 *__restrict__ block_sums) {
    int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint2 acc = make_uint2(0, 0);
    for (int i = 0; i < kScanItems; ++i) acc = add2(acc, pair_of(hist, base + i, n, R));
    uint2 total;
    block_exclusive_scan(acc, &total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Single-block exclusive scan of the block sums (in place); writes the grand
// total to *total.
__global__ __launch_bounds__(256) void scan_sums_kernel(uint2 *__restrict__ sums, int64_t nb,
                                                        uint2 *__restrict__ total) {
    uint2 carry = make_uint2(0, 0);
    for (int64_t base = 0; base < nb; base += 256) {
        int64_t i = base + threadIdx.x;
        uint2 v = (i < nb) ? sums[i] : make_uint2(0, 0);
        uint2 tot;
        uint2 ex = block_exclusive_scan(v, &tot);
        if (i < nb) sums[i] = add2(ex, carry);
        carry = add2(carry, tot);
    }
    if (threadIdx.x == 0) *total = carry;
}

// Writes bstart[i] (first record of bucket i), cursor[i] (= bstart, used by
// the scatter) and cstart[i] (first chunk of bucket i).
__global__ __launch_bounds__(256) void scan_down_kernel(const uint32_t *__restrict__ hist,
                                                        int64_t n, uint32_t R,
                                                        const uint2 *__restrict__ block_off,
                                                        uint32_t *__restrict__ bstart,
                                                        uint32_t *__restrict__ cursor,
                                                        uint32_t *__restrict__ cstart) {
    int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint2 vals[kScanItems];
    uint2 acc = make_uint2(0, 0);
    for (int i = 0; i < kScanItems; ++i) {
        vals[i] = pair_of(hist, base + i, n, R);
        acc = add2(acc, vals[i]);
    }
    uint2 total;
    uint2 run = add2(block_exclusive_scan(acc, &total), block_off[blockIdx.x]);
    for (int i = 0; i < kScanItems; ++i) {
        int64_t k = base + i;
        if (k < n) {
            bstart[k] = run.x;
            cursor[k] = run.x;
            cstart[k] = run.y;
        }
        run = add2(run, vals[i]);
    }
}

// ---------------------------------------------------------------------------
// scatter records into bucket order (order inside a bucket is arbitrary;
// the chunk sort below orders each chunk by cell)
// ---------------------------------------------------------------------------
// Valid records go to their bucket's slots; skipped records follow all valid
// ones (sperm only: their outputs are zeroed by the degridder).
template <typename T>
__global__ __launch_bounds__(256) void scatter_kernel(DevGeom g,
                                                      const PlaneLayout *__restrict__ planes,
                                                      int64_t nrec, const T *__restrict__ uvw,
                                                      uint32_t *__restrict__ cursor,
                                                      const uint2 *__restrict__ total,
                                                      int64_t *__restrict__ counters,
                                                      RecMeta *__restrict__ smeta,
                                                      uint32_t *__restrict__ sperm) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
    const int64_t nvalid = (int64_t)total->x;
    for (int64_t r0 = first; r0 < nrec; r0 += stride) {
        const int64_t r = r0 + (threadIdx.x & 63);
        uint32_t b = kInvalidBucket;
        RecIndex ix;
        if (r < nrec) ix = index_bucket<T>(g, planes, uvw, r, &b);
        const bool act = b != kInvalidBucket;
        const uint32_t pos = wave_counter_add(cursor, b, act, true);
        if (act) {
            smeta[pos] = pack_meta(g, ix);
            sperm[pos] = (uint32_t)r;
        } else if (r < nrec) {
            const int64_t q = nvalid + (int64_t)atomicAdd((unsigned long long *)&counters[3], 1ull);
            if (q < nrec) sperm[q] = (uint32_t)r;
        }
    }
}

// ---------------------------------------------------------------------------
// chunk list: bucket b with c records -> ceil(c/R) chunks
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void chunk_list_kernel(int64_t nb, uint32_t R,
                                                         const uint32_t *__restrict__ hist,
                                                         const uint32_t *__restrict__ bstart,
                                                         const uint32_t *__restrict__ cstart,
                                                         Chunk *__restrict__ chunks) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x) {
        uint32_t c = hist[b];
        uint32_t s = bstart[b];
        uint32_t k0 = cstart[b];
        for (uint32_t k = 0; k * R < c; ++k) {
            Chunk ch;
            ch.start = s + k * R;
            ch.len = min(R, c - k * R);
            ch.bucket = (uint32_t)b;
            ch.bbox = 0;
            chunks[k0 + k] = ch;
        }
    }
}

// plane_cfirst[p] = first chunk of plane p; plane_cfirst[P] = chunk count.
// counters[1] = valid records, counters[2] = chunks (counters[3] counts the
// skipped records placed by the scatter).
__global__ void plane_ranges_kernel(int32_t nplanes, const PlaneLayout *__restrict__ planes,
                                    int64_t nb, uint32_t *__restrict__ cstart,
                                    const uint2 *__restrict__ total,
                                    uint32_t *__restrict__ plane_cfirst,
                                    int64_t *__restrict__ counters) {
    for (int p = threadIdx.x; p < nplanes; p += blockDim.x)
        plane_cfirst[p] = (planes[p].base < nb) ? cstart[planes[p].base] : total->y;
    if (threadIdx.x == 0) {
        plane_cfirst[nplanes] = total->y;
        cstart[nb] = total->y;   // end of the last bucket's chunks
        counters[1] = total->x;
        counters[2] = total->y;
    }
}

// ---------------------------------------------------------------------------
// units of a plane group: the chunks of one tile, over
// all planes of the group, split greedily into runs of at most `cap`
// records (a chunk is never split).  The gridders take a unit at a time
// and commit the tile's region once per unit rather than once per chunk.  units[first chunk of the group + k] = (first chunk, chunk count)
// of the group's unit k; group_nunits[g] = unit count (cleared beforehand).
// A wave's units are consecutive and in tile order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void unit_list_kernel(const PlaneLayout *__restrict__ planes,
                                                        int32_t g,
                                                        const uint32_t *__restrict__ bucket_cfirst,
                                                        const Chunk *__restrict__ chunks,
                                                        uint32_t cap, uint2 *__restrict__ units,
                                                        uint32_t *__restrict__ group_nunits) {
    const PlaneLayout pl = planes[g];
    const uint32_t ntiles = (uint32_t)pl.ntu * (uint32_t)pl.ntv;
    const uint32_t n = (uint32_t)pl.grp_n;
    const int64_t base = pl.base;
    const int lane = threadIdx.x & 63;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t cs = 0, ce = 0;
    if (t < ntiles) {
        cs = bucket_cfirst[base + (int64_t)t * n];
        ce = bucket_cfirst[base + (int64_t)(t + 1) * n];
    }
    // A bucket's chunks are full (cap records) but for its last one, so the
    // greedy split only has to look at each bucket's chunk count and last
    // length: full chunks are units of their own, and a bucket's last chunk
    // joins the open unit if it fits (acc = cap opens a unit at the first
    // chunk).
    auto walk = [&](auto emit) {
        uint32_t acc = cap, head = cs;
        for (uint32_t j = 0; j < n && cs < ce; ++j) {
            const int64_t b = base + (int64_t)t * n + j;
            const uint32_t b0 = bucket_cfirst[b], b1 = bucket_cfirst[b + 1];
            if (b0 == b1) continue;
            const uint32_t last_len = chunks[b1 - 1].len;
            for (uint32_t c = b0; c + 1 < b1; ++c) {   // full chunks
                if (c > head) emit(head, c);
                head = c;
                acc = cap;
            }
            if (acc + last_len > cap) {
                if (b1 - 1 > head) emit(head, b1 - 1);
                head = b1 - 1;
                acc = last_len;
            } else {
                acc += last_len;
            }
        }
        if (ce > cs) emit(head, ce);
    };
    // pass 1: unit count of this tile
    uint32_t cnt = 0;
    walk([&](uint32_t, uint32_t) { ++cnt; });
    // wave prefix sum; one lane reserves the wave's units
    uint32_t incl = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
    }
    const uint32_t wtotal = __shfl(incl, 63, 64);
    uint32_t wbase = 0;
    if (lane == 63 && wtotal) wbase = atomicAdd(&group_nunits[g], wtotal);
    wbase = __shfl(wbase, 63, 64);
    // pass 2: write them
    uint2 *out = units + bucket_cfirst[base] + wbase + (incl - cnt);
    walk([&](uint32_t h, uint32_t e) { *out++ = make_uint2(h, e - h); });
}

// ---------------------------------------------------------------------------
// per-chunk counting sort by cell inside the tile, in LDS: column by column
// (u outer), v running up and down in alternate columns, so consecutive
// records step by one cell and a moving window retires one row or column of
// slots at a time (a plain column-major order would retire most slots at
// every column change)
// ---------------------------------------------------------------------------
constexpr int kMaxR = 2048;

__device__ inline uint32_t cell_key(uint32_t du, uint32_t dv, int log2T) {
    const uint32_t vv = (du & 1u) ? ((1u << log2T) - 1u - dv) : dv;
    return (du << log2T) | vv;
}


// Chunks of at most kWaveSortMax records: one wave per chunk sorts the
// (cell key, lane) pairs with a bitonic network across its lanes, then each
// lane fetches the record of its rank; no LDS and no barriers.  Larger
// chunks take the workgroup counting sort below.
constexpr uint32_t kWaveSortMax = 64;

__global__ __launch_bounds__(256) void chunk_sort_small_kernel(
    const uint32_t *__restrict__ plane_cfirst, int32_t nplanes,
    const PlaneLayout *__restrict__ planes, Chunk *__restrict__ chunks,
    RecMeta *__restrict__ smeta, uint32_t *__restrict__ sperm) {
    const uint32_t c_end = plane_cfirst[nplanes];
    const int lane = threadIdx.x & 63;
    const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
    int p = 0;   // chunks come in increasing order: the plane only moves forward
    for (uint32_t c = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); c < c_end;
         c += nwaves) {
        const Chunk ch = chunks[c];
        if (ch.len > kWaveSortMax) continue;
        while (p + 1 < nplanes && c >= plane_cfirst[p + 1]) ++p;
        int pp;
        uint32_t tile;
        bucket_plane_tile(planes[p], ch.bucket, &pp, &tile);
        const PlaneLayout pl = planes[pp];
        if (pl.cls >= 3) continue;   // the blocked kernels need neither
        const uint32_t tu0 = (tile % (uint32_t)pl.ntu) << pl.log2T;
        const uint32_t tv0 = (tile / (uint32_t)pl.ntu) << pl.log2T;
        RecMeta m{0u, 0u};
        uint32_t perm = 0u;
        uint32_t v = 0xffffffffu;   // lanes past the chunk sort last
        uint32_t umin = 0xffu, umax = 0u, vmin = 0xffu, vmax = 0u;
        if ((uint32_t)lane < ch.len) {
            m = smeta[ch.start + lane];
            perm = sperm[ch.start + lane];
            const uint32_t du = meta_ku(m) - tu0, dv = meta_kv(m) - tv0;
            v = (cell_key(du, dv, pl.log2T) << 6) | (uint32_t)lane;
            umin = umax = du;
            vmin = vmax = dv;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            umin = min(umin, (uint32_t)__shfl_xor((int)umin, off, 64));
            umax = max(umax, (uint32_t)__shfl_xor((int)umax, off, 64));
            vmin = min(vmin, (uint32_t)__shfl_xor((int)vmin, off, 64));
            vmax = max(vmax, (uint32_t)__shfl_xor((int)vmax, off, 64));
        }
        if (lane == 0) chunks[c].bbox = umin | (umax << 8) | (vmin << 16) | (vmax << 24);
        if (ch.len < 2) continue;
#pragma unroll
        for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                const uint32_t o = (uint32_t)__shfl_xor((int)v, j, 64);
                const bool take_min = ((lane & j) == 0) == ((lane & k) == 0);
                v = take_min ? min(v, o) : max(v, o);
            }
        }
        const int src = (int)(v & 63u);
        const uint32_t kuv = (uint32_t)__shfl((int)m.kuv, src, 64);
        const uint32_t toff = (uint32_t)__shfl((int)m.toff, src, 64);
        const uint32_t pr = (uint32_t)__shfl((int)perm, src, 64);
        if ((uint32_t)lane < ch.len) {
            smeta[ch.start + lane] = RecMeta{kuv, toff};
            sperm[ch.start + lane] = pr;
        }
    }
}

__global__ __launch_bounds__(256) void chunk_sort_kernel(const uint32_t *__restrict__ plane_cfirst,
                                                         int32_t nplanes,
                                                         const PlaneLayout *__restrict__ planes,
                                                         Chunk *__restrict__ chunks,
                                                         RecMeta *__restrict__ smeta,
                                                         uint32_t *__restrict__ sperm) {
    __shared__ uint32_t hist[1024];
    __shared__ RecMeta m_in[kMaxR];
    __shared__ uint32_t p_in[kMaxR];
    __shared__ uint32_t s_box[4][4];   // per wave: umin, umax, vmin, vmax
    // only chunks of supports up to 32 are cell-sorted and bounded; the
    // blocked kernels of the larger supports take the records in any order
    const uint32_t c_end = plane_cfirst[nplanes];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int p = 0;   // chunks come in increasing order: the plane only moves forward
    for (uint32_t c = blockIdx.x; c < c_end; c += gridDim.x) {
        const Chunk ch = chunks[c];
        if (ch.len <= kWaveSortMax) continue;   // the wave sort's chunks
        while (p + 1 < nplanes && c >= plane_cfirst[p + 1]) ++p;
        int pp;
        uint32_t tile;
        bucket_plane_tile(planes[p], ch.bucket, &pp, &tile);
        const PlaneLayout pl = planes[pp];
        if (pl.cls >= 3) continue;
        const uint32_t tu0 = (tile % (uint32_t)pl.ntu) << pl.log2T;
        const uint32_t tv0 = (tile / (uint32_t)pl.ntu) << pl.log2T;
        const int ncell = pl.T * pl.T;
        for (int i = threadIdx.x; i < ncell; i += blockDim.x) hist[i] = 0;
        __syncthreads();
        uint32_t umin = 0xffu, umax = 0u, vmin = 0xffu, vmax = 0u;
        for (uint32_t i = threadIdx.x; i < ch.len; i += blockDim.x) {
            RecMeta m = smeta[ch.start + i];
            m_in[i] = m;
            p_in[i] = sperm[ch.start + i];
            uint32_t du = meta_ku(m) - tu0, dv = meta_kv(m) - tv0;
            atomicAdd(&hist[cell_key(du, dv, pl.log2T)], 1u);
            umin = min(umin, du);
            umax = max(umax, du);
            vmin = min(vmin, dv);
            vmax = max(vmax, dv);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            umin = min(umin, (uint32_t)__shfl_xor((int)umin, off, 64));
            umax = max(umax, (uint32_t)__shfl_xor((int)umax, off, 64));
            vmin = min(vmin, (uint32_t)__shfl_xor((int)vmin, off, 64));
            vmax = max(vmax, (uint32_t)__shfl_xor((int)vmax, off, 64));
        }
        if (lane == 0) {
            s_box[wave][0] = umin;
            s_box[wave][1] = umax;
            s_box[wave][2] = vmin;
            s_box[wave][3] = vmax;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < 4; ++w) {
                umin = min(umin, s_box[w][0]);
                umax = max(umax, s_box[w][1]);
                vmin = min(vmin, s_box[w][2]);
                vmax = max(vmax, s_box[w][3]);
            }
            chunks[c].bbox = umin | (umax << 8) | (vmin << 16) | (vmax << 24);
        }
        {
            // exclusive scan of the (up to 1024) cell counts: 4 per thread
            uint2 v = make_uint2(0, 0);
            uint32_t loc[4];
            for (int k = 0; k < 4; ++k) {
                int i = threadIdx.x * 4 + k;
                loc[k] = (i < ncell) ? hist[i] : 0u;
                v.x += loc[k];
            }
            uint2 tot;
            uint2 ex = block_exclusive_scan(v, &tot);
            uint32_t run = ex.x;
            for (int k = 0; k < 4; ++k) {
                int i = threadIdx.x * 4 + k;
                if (i < ncell) hist[i] = run;
                run += loc[k];
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < ch.len; i += blockDim.x) {
            RecMeta m = m_in[i];
            uint32_t du = meta_ku(m) - tu0, dv = meta_kv(m) - tv0;
            uint32_t pos = atomicAdd(&hist[cell_key(du, dv, pl.log2T)], 1u);
            smeta[ch.start + pos] = m;
            sperm[ch.start + pos] = p_in[i];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// compute_indices: the index rule written out per record (parity/debug)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void indices_kernel(DevGeom g, int64_t nrec,
                                                      const T *__restrict__ uvw,
                                                      int32_t *k_lo_u, int32_t *k_lo_v,
                                                      int32_t *o_u, int32_t *o_v, int32_t *plane,
                                                      uint8_t *valid, int64_t *d_nskipped) {
    __shared__ uint32_t s_skip;
    if (threadIdx.x == 0) s_skip = 0;
    __syncthreads();
    uint32_t skipped = 0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrec;
         r += (int64_t)gridDim.x * blockDim.x) {
        // k_lo and o are 0 for skipped records
        RecIndex ix = index_record<T>(g, uvw[3 * r], uvw[3 * r + 1], uvw[3 * r + 2]);
        k_lo_u[r] = ix.ku;
        k_lo_v[r] = ix.kv;
        o_u[r] = ix.ou;
        o_v[r] = ix.ov;
        plane[r] = ix.plane;
        valid[r] = (uint8_t)ix.valid;
        skipped += !ix.valid;
    }
    if (d_nskipped) {
        if (skipped) atomicAdd(&s_skip, skipped);
        __syncthreads();
        if (threadIdx.x == 0 && s_skip)
            atomicAdd((unsigned long long *)d_nskipped, (unsigned long long)s_skip);
    }
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int grid_blocks(int64_t n, int threads) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (int)b;
}

// The plan's tap table, phase-major (see common.h): entry
// (o_v, o_u, j, i) of plane p takes bank element (o_v + 1 + j beta) *
// (beta S + 1) + (o_u + 1 + i beta) of the caller's plane; for W-projection
// (complex entries, (re, im) pairs of T) its conjugate also goes to
// conj_base + the same index.  Separable: entry (o, i) takes o + 1 + i beta.
// Also raises planes[p].tmax to the largest |component| copied (the plane
// layouts arrive with tmax = 0; non-negative floats order like their bits).
template <typename T>
__global__ __launch_bounds__(256) void tap_layout_kernel(PlaneLayout *__restrict__ planes,
                                                         int32_t beta, int32_t wproj,
                                                         const T *__restrict__ src,
                                                         T *__restrict__ dst, int64_t conj_base) {
    const PlaneLayout pl = planes[blockIdx.y];
    const int64_t S = pl.S;
    const int64_t ws = (int64_t)beta * S + 1;   // caller's row length
    const int64_t n = wproj ? (int64_t)beta * beta * S * S : (int64_t)beta * S;
    float m = 0.0f;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % S;
        const int64_t d = (int64_t)pl.tap_off + e;
        if (wproj) {
            const int64_t blk = e / (S * S);
            const int64_t j = (e / S) % S;
            const int64_t ou = blk % beta, ov = blk / beta;
            const int64_t sidx = (int64_t)pl.src_off + (ov + 1 + j * beta) * ws + (ou + 1 + i * beta);
            const T re = src[2 * sidx], im = src[2 * sidx + 1];
            dst[2 * d] = re;
            dst[2 * d + 1] = im;
            dst[2 * (conj_base + d)] = re;
            dst[2 * (conj_base + d) + 1] = -im;
            m = fmaxf(m, fmaxf(fabsf(TapTraits<T>::real(&re, 0)), fabsf(TapTraits<T>::real(&im, 0))));
        } else {
            const int64_t o = e / S;
            const T t = src[o + 1 + i * beta];
            dst[d] = t;
            m = fmaxf(m, fabsf(TapTraits<T>::real(&t, 0)));
        }
    }
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0 && m > 0.0f)
        atomicMax(reinterpret_cast<unsigned int *>(&planes[blockIdx.y].tmax), __float_as_uint(m));
}

}  // namespace

mg_status plan_taps(PlanState &P, const void *src, int64_t table_elems, hipStream_t stream) {
    const int np = P.nplanes_eff;
    const bool wproj = P.kind == MG_KERNEL_WPROJ;
    hipError_t e = hipMemcpyAsync(P.d_planes, P.planes.data(), sizeof(PlaneLayout) * np,
                                  hipMemcpyHostToDevice, stream);
    if (e != hipSuccess)
        return set_error(MG_EDEVICE, std::string("plane layout upload: ") + hipGetErrorString(e));
    int64_t most = 0;
    for (const PlaneLayout &L : P.planes) {
        const int64_t w = (int64_t)P.geom.beta * L.S;
        most = std::max<int64_t>(most, wproj ? w * w : w);
    }
    const dim3 grid((unsigned)std::min<int64_t>(grid_blocks(most, 256), 1024), (unsigned)np);
    const int32_t beta = P.geom.beta;
    if (P.tap_dtype == MG_F16)
        hipLaunchKernelGGL(tap_layout_kernel<__half>, grid, dim3(256), 0, stream, P.d_planes, beta,
                           (int32_t)wproj, (const __half *)src, (__half *)P.taps, table_elems);
    else if (P.tap_dtype == MG_BF16)
        hipLaunchKernelGGL(tap_layout_kernel<__hip_bfloat16>, grid, dim3(256), 0, stream,
                           P.d_planes, beta, (int32_t)wproj, (const __hip_bfloat16 *)src,
                           (__hip_bfloat16 *)P.taps, table_elems);
    else
        hipLaunchKernelGGL(tap_layout_kernel<float>, grid, dim3(256), 0, stream, P.d_planes, beta,
                           (int32_t)wproj, (const float *)src, (float *)P.taps, table_elems);
    e = hipGetLastError();
    if (e != hipSuccess) return set_error(MG_EDEVICE, std::string("tap layout: ") + hipGetErrorString(e));
    return MG_OK;
}

mg_status launch_compute_indices(const DevGeom &g, int64_t nrec, const void *uvw,
                                 mg_dtype uvw_dtype, int32_t *k_lo_u, int32_t *k_lo_v,
                                 int32_t *o_u, int32_t *o_v, int32_t *plane, uint8_t *valid,
                                 int64_t *d_nskipped, hipStream_t stream) {
    if (nrec == 0) return MG_OK;
    int nb = grid_blocks(nrec, 256);
    if (uvw_dtype == MG_F32)
        hipLaunchKernelGGL(indices_kernel<float>, dim3(nb), dim3(256), 0, stream, g, nrec,
                           (const float *)uvw, k_lo_u, k_lo_v, o_u, o_v, plane, valid, d_nskipped);
    else
        hipLaunchKernelGGL(indices_kernel<double>, dim3(nb), dim3(256), 0, stream, g, nrec,
                           (const double *)uvw, k_lo_u, k_lo_v, o_u, o_v, plane, valid,
                           d_nskipped);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(MG_EDEVICE, std::string("index kernel: ") + hipGetErrorString(e));
    return MG_OK;
}

mg_status plan_build(PlanState &P, const void *uvw, mg_dtype uvw_dtype, hipStream_t stream) {
    const int64_t nrec = P.nrec;
    const int64_t nb = P.nbuckets;
    const uint32_t R = (uint32_t)P.R;
    const int np = P.nplanes_eff;
    hipError_t e = hipSuccess;
    uint32_t *hist = P.hist, *bstart = P.bstart, *cursor = P.cursor;
    uint32_t *cstart = P.bucket_cfirst;   // kept: first chunk of each bucket
    uint2 *sums = P.sums;
    const int64_t nscan = (nb + kScanBlock - 1) / kScanBlock;

    // zero-fill with a kernel (no memset nodes, so the calls stay capturable)
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(256), 0, stream, (uint32_t *)P.counters,
                       (int64_t)12, 0u);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_blocks(nb, 256)), dim3(256), 0, stream, hist,
                       nb, 0u);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(256), 0, stream, P.group_nunits,
                       (int64_t)np, 0u);
    if (nrec > 0) {
        int g1 = grid_blocks(nrec, 256);
        if (uvw_dtype == MG_F32)
            hipLaunchKernelGGL(index_bucket_kernel<float>, dim3(g1), dim3(256), 0, stream, P.geom,
                               P.d_planes, nrec, (const float *)uvw, hist, P.counters);
        else
            hipLaunchKernelGGL(index_bucket_kernel<double>, dim3(g1), dim3(256), 0, stream,
                               P.geom, P.d_planes, nrec, (const double *)uvw, hist, P.counters);
    }
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nscan), dim3(256), 0, stream, hist, nb,
                       R, sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(256), 0, stream, sums, nscan, sums + nscan);
    hipLaunchKernelGGL(scan_down_kernel, dim3((unsigned)nscan), dim3(256), 0, stream, hist, nb, R,
                       sums, bstart, cursor, cstart);
    if (nrec > 0) {
        const dim3 g1(grid_blocks(nrec, 256));
        if (uvw_dtype == MG_F32)
            hipLaunchKernelGGL(scatter_kernel<float>, g1, dim3(256), 0, stream, P.geom, P.d_planes,
                               nrec, (const float *)uvw, cursor, sums + nscan, P.counters, P.smeta,
                               P.sperm);
        else
            hipLaunchKernelGGL(scatter_kernel<double>, g1, dim3(256), 0, stream, P.geom,
                               P.d_planes, nrec, (const double *)uvw, cursor, sums + nscan,
                               P.counters, P.smeta, P.sperm);
    }
    hipLaunchKernelGGL(chunk_list_kernel, dim3(grid_blocks(nb, 256)), dim3(256), 0, stream, nb, R,
                       hist, bstart, cstart, P.chunks);
    hipLaunchKernelGGL(plane_ranges_kernel, dim3(1), dim3(256), 0, stream, np, P.d_planes, nb,
                       cstart, sums + nscan, P.plane_cfirst, P.counters);
    {
        // cell sort and bounding box of the chunks of the window gridders'
        // supports (up to 32): small chunks one per wave, the others one per
        // workgroup
        hipLaunchKernelGGL(chunk_sort_small_kernel, dim3(8 * device_cus()), dim3(256), 0,
                           stream, P.plane_cfirst, np, P.d_planes, P.chunks, P.smeta, P.sperm);
        hipLaunchKernelGGL(chunk_sort_kernel,
                           dim3(resident_groups((const void *)chunk_sort_kernel, 256, 0)),
                           dim3(256), 0, stream, P.plane_cfirst, np, P.d_planes, P.chunks,
                           P.smeta, P.sperm);
        // units of every plane group
        for (int p = 0; p < np; p += P.planes[p].grp_n) {
            const PlaneLayout &L = P.planes[p];
            const int64_t ntiles = (int64_t)L.ntu * L.ntv;
            hipLaunchKernelGGL(unit_list_kernel, dim3(grid_blocks(ntiles, 256)), dim3(256), 0,
                               stream, P.d_planes, p, P.bucket_cfirst, P.chunks, R, P.units,
                               P.group_nunits);
        }
    }
    e = hipGetLastError();
    if (e != hipSuccess) return set_error(MG_EDEVICE, std::string("plan kernels: ") + hipGetErrorString(e));
    return MG_OK;
}

// Arena layout of a plan: every array starts on a kArenaAlign boundary.
namespace {
template <typename F>
size_t walk_arena(const PlanState &P, F &&place) {
    const int np = P.nplanes_eff;
    const int64_t nb = P.nbuckets;
    const int64_t nscan = (nb + kScanBlock - 1) / kScanBlock;
    const size_t n = (size_t)(P.nrec + kRecPad);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += arena_round(bytes);
        return at;
    };
    place(0, take(sizeof(PlaneLayout) * (size_t)np));
    place(1, take(P.taps_bytes));
    place(2, take(sizeof(RecMeta) * n));
    place(3, take(sizeof(uint32_t) * n));
    place(4, take(sizeof(Chunk) * (size_t)P.max_chunks));
    place(5, take(sizeof(uint32_t) * (size_t)(np + 1)));
    place(6, take(sizeof(uint32_t) * (size_t)(nb + 1)));
    place(7, take(sizeof(uint2) * (size_t)P.max_chunks));
    place(8, take(sizeof(uint32_t) * (size_t)np));
    place(9, take(sizeof(int64_t) * 6));
    place(10, take(sizeof(uint32_t) * (size_t)nb));
    place(11, take(sizeof(uint32_t) * (size_t)nb));
    place(12, take(sizeof(uint32_t) * (size_t)nb));
    place(13, take(sizeof(uint2) * (size_t)(nscan + 1)));
    return off;
}
}  // namespace

size_t plan_arena_bytes(const PlanState &P) {
    return walk_arena(P, [](int, size_t) {});
}

void plan_carve(PlanState &P, void *arena) {
    char *base = static_cast<char *>(arena);
    P.bytes = walk_arena(P, [&](int what, size_t at) {
        void *p = base + at;
        switch (what) {
        case 0: P.d_planes = static_cast<PlaneLayout *>(p); break;
        case 1: P.taps = p; break;
        case 2: P.smeta = static_cast<RecMeta *>(p); break;
        case 3: P.sperm = static_cast<uint32_t *>(p); break;
        case 4: P.chunks = static_cast<Chunk *>(p); break;
        case 5: P.plane_cfirst = static_cast<uint32_t *>(p); break;
        case 6: P.bucket_cfirst = static_cast<uint32_t *>(p); break;
        case 7: P.units = static_cast<uint2 *>(p); break;
        case 8: P.group_nunits = static_cast<uint32_t *>(p); break;
        case 9: P.counters = static_cast<int64_t *>(p); break;
        case 10: P.hist = static_cast<uint32_t *>(p); break;
        case 11: P.bstart = static_cast<uint32_t *>(p); break;
        case 12: P.cursor = static_cast<uint32_t *>(p); break;
        default: P.sums = static_cast<uint2 *>(p); break;
        }
    });
}

}  // namespace mg
