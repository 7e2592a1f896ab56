// Hybrid Gridding Step and column pruning.
//
// Hybrid Gridding (Algorithm "The studied Hybrid Gridding Algorithm",
// Section 2.4.4) splits the Gridding Step of convolutional gridding in one
// dimension: along u a record is convolved with the oversampled separable
// kernel (S taps at the integer cells, the same rule as the convolutional
// gridder), along v it is moved to the nearest pixel of the beta-oversampled
// v axis (nearest-neighbour interpolation, C_hy = C_co(u) rect(v)).  The
// output is an nu x (beta nv) grid per polarisation, [npol][beta nv][nu],
// origin at column nu/2, row beta nv / 2.  A record updates S cells of one
// row instead of S^2 cells.  The Pruning Step then downsamples every column
// by alpha with a convolution (Convolution-Based FFT Pruning, Section 2.5.2;
// the Column Pruner of Section 7.1).
//
// gfx950 design.
//  * Plan (sort once, grid many times): records are binned by tile of 32
//    columns x 32 oversampled rows and cut into chunks of at most R records;
//    each record keeps (k_lo_u | o_u << 16, row) and its input index.
//  * Gridder: a workgroup takes a chunk.  Its records' S x 1 footprints lie
//    in the tile's region (32 rows x (31 + S) columns), accumulated in LDS as
//    32-bit fixed point, like the window gridders' regions: the chunk first
//    bounds its partial sums (2 max|tap| sum over its records of the largest
//    visibility component), picks the power-of-two scale that maps the bound
//    to at most 2^30, and every update is one rounded conversion and one
//    integer LDS atomic.  Lane l of a wave takes component c = l mod 8
//    (polarisation c/2, real or imaginary part) of tap i = l / 8 of the
//    wave's record, so a record's S x 8 updates are one wave instruction for
//    S <= 8 (consecutive LDS words: no bank conflicts).  At the end of the
//    chunk the region is added to the grid with one float atomic per touched
//    word.  A chunk holding a non-finite visibility (or whose bound
//    overflows) adds straight to the grid in FP32.
//  * Column pruner: one thread per (polarisation, column) and run of output
//    rows keeps S_z accumulators in registers as a ring (the chunk
//    calculation of Section 7.1.5): every input value is read once, with
//    coalesced rows, and multiplied by the S_z coefficients its offset
//    needs, which are uniform across the wave (scalar operands).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace mg {

namespace {

constexpr int kHyTU = 32;          // tile columns (u cells)
constexpr int kHyTV = 16;          // tile rows (rows of the oversampled v axis)
constexpr int kHyThreads = 256;
constexpr int kHyMaxS = 32;
constexpr int kHyWaves = kHyThreads / kWave;

struct HyGeom {
    int32_t nu, nv, npol, beta, S;
    int32_t ntu, ntv;              // tiles per axis
    int32_t rows;                  // beta * nv
    double scale_u, scale_v;
};

// The hybrid index rule: the u axis as the convolutional gridder (first cell
// k_lo_u, phase o_u), the v axis the nearest pixel of the beta-oversampled
// axis, q = floor(beta x_v + 1/2), each operation rounded as written.
template <typename T>
__device__ inline bool hy_index(const HyGeom &g, T u_, T v_, T w_, int32_t *ku, int32_t *ou,
                                int32_t *q) {
#pragma clang fp contract(off)
    const double u = (double)u_, v = (double)v_, w = (double)w_;
    if (!(isfinite(u) && isfinite(v) && isfinite(w))) return false;
    if (!index_axis(u, g.scale_u, g.nu, g.beta, g.S, ku, ou)) return false;
    double x = v * g.scale_v;
    x = x + (double)(g.nv / 2);
    double xb = x * (double)g.beta;
    xb = xb + 0.5;
    const double fq = floor(xb);
    if (!(fq >= 0.0) || !(fq < (double)g.rows)) return false;
    *q = (int32_t)fq;
    return true;
}

__device__ inline uint32_t hy_bucket(const HyGeom &g, int32_t ku, int32_t q) {
    return (uint32_t)(q / kHyTV) * (uint32_t)g.ntu + (uint32_t)(ku / kHyTU);
}

constexpr uint32_t kNoBucket = 0xffffffffu;

template <typename T>
__global__ __launch_bounds__(256) void hy_count_kernel(HyGeom g, int64_t nrec,
                                                       const T *__restrict__ uvw,
                                                       uint32_t *__restrict__ hist,
                                                       int64_t *__restrict__ counters) {
    __shared__ uint32_t s_skip;
    if (threadIdx.x == 0) s_skip = 0;
    __syncthreads();
    uint32_t skipped = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
    for (int64_t r0 = first; r0 < nrec; r0 += stride) {
        const int64_t r = r0 + (threadIdx.x & 63);
        uint32_t b = kNoBucket;
        if (r < nrec) {
            int32_t ku, ou, q;
            if (hy_index<T>(g, uvw[3 * r], uvw[3 * r + 1], uvw[3 * r + 2], &ku, &ou, &q))
                b = hy_bucket(g, ku, q);
            else
                ++skipped;
        }
        wave_counter_add(hist, b, b != kNoBucket, false);
    }
    if (skipped) atomicAdd(&s_skip, skipped);
    __syncthreads();
    if (threadIdx.x == 0 && s_skip)
        atomicAdd((unsigned long long *)&counters[0], (unsigned long long)s_skip);
}

// Exclusive scan of the bucket counts and of their chunk counts (ceil(c/R)),
// one workgroup: bstart, cursor (= bstart), cstart; counters[1] = valid
// records, counters[2] = chunks.
__global__ __launch_bounds__(256) void hy_scan_kernel(const uint32_t *__restrict__ hist, int64_t nb,
                                                      uint32_t R, uint32_t *__restrict__ bstart,
                                                      uint32_t *__restrict__ cursor,
                                                      uint32_t *__restrict__ cstart,
                                                      int64_t *__restrict__ counters) {
    constexpr int kItems = 16;
    __shared__ uint32_t s_rec[256], s_chk[256];
    uint32_t carry_r = 0, carry_c = 0;
    for (int64_t base = 0; base < nb; base += 256 * kItems) {
        uint32_t cr[kItems], cc[kItems];
        uint32_t tr = 0, tc = 0;
        const int64_t b0 = base + (int64_t)threadIdx.x * kItems;
        for (int k = 0; k < kItems; ++k) {
            const uint32_t c = (b0 + k < nb) ? hist[b0 + k] : 0u;
            cr[k] = c;
            cc[k] = (c + R - 1) / R;
            tr += cr[k];
            tc += cc[k];
        }
        s_rec[threadIdx.x] = tr;
        s_chk[threadIdx.x] = tc;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const uint32_t ar = (threadIdx.x >= (unsigned)off) ? s_rec[threadIdx.x - off] : 0u;
            const uint32_t ac = (threadIdx.x >= (unsigned)off) ? s_chk[threadIdx.x - off] : 0u;
            __syncthreads();
            s_rec[threadIdx.x] += ar;
            s_chk[threadIdx.x] += ac;
            __syncthreads();
        }
        uint32_t run_r = carry_r + s_rec[threadIdx.x] - tr;
        uint32_t run_c = carry_c + s_chk[threadIdx.x] - tc;
        for (int k = 0; k < kItems; ++k) {
            if (b0 + k < nb) {
                bstart[b0 + k] = run_r;
                cursor[b0 + k] = run_r;
                cstart[b0 + k] = run_c;
            }
            run_r += cr[k];
            run_c += cc[k];
        }
        carry_r += s_rec[255];
        carry_c += s_chk[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cstart[nb] = carry_c;
        counters[1] = carry_r;
        counters[2] = carry_c;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void hy_scatter_kernel(HyGeom g, int64_t nrec,
                                                         const T *__restrict__ uvw,
                                                         uint32_t *__restrict__ cursor,
                                                         uint2 *__restrict__ meta,
                                                         uint32_t *__restrict__ perm) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
    for (int64_t r0 = first; r0 < nrec; r0 += stride) {
        const int64_t r = r0 + (threadIdx.x & 63);
        uint32_t b = kNoBucket;
        int32_t ku = 0, ou = 0, q = 0;
        if (r < nrec && hy_index<T>(g, uvw[3 * r], uvw[3 * r + 1], uvw[3 * r + 2], &ku, &ou, &q))
            b = hy_bucket(g, ku, q);
        const bool act = b != kNoBucket;
        const uint32_t pos = wave_counter_add(cursor, b, act, true);
        if (act) {
            meta[pos] = make_uint2((uint32_t)ku | ((uint32_t)ou << 16), (uint32_t)q);
            perm[pos] = (uint32_t)r;
        }
    }
}

__global__ __launch_bounds__(256) void hy_chunks_kernel(int64_t nb, uint32_t R,
                                                        const uint32_t *__restrict__ hist,
                                                        const uint32_t *__restrict__ bstart,
                                                        const uint32_t *__restrict__ cstart,
                                                        Chunk *__restrict__ chunks) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = hist[b], s = bstart[b], k0 = cstart[b];
        for (uint32_t k = 0; k * R < c; ++k)
            chunks[k0 + k] = Chunk{s + k * R, min(R, c - k * R), (uint32_t)b, 0u};
    }
}

// The plan's tap table as FP32, phase-major (entry o S + i = caller's entry
// o + 1 + i beta), and the largest |tap| (non-negative floats order like
// their bits).
template <typename TapT>
__global__ __launch_bounds__(256) void hy_taps_kernel(int32_t beta, int32_t S,
                                                      const TapT *__restrict__ src,
                                                      float *__restrict__ dst,
                                                      float *__restrict__ tmax) {
    float m = 0.0f;
    for (int e = threadIdx.x; e < beta * S; e += blockDim.x) {
        const int o = e / S, i = e % S;
        const float t = TapTraits<TapT>::real(src, (int64_t)o + 1 + (int64_t)i * beta);
        dst[e] = t;
        m = fmaxf(m, fabsf(t));
    }
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(reinterpret_cast<unsigned int *>(tmax), __float_as_uint(m));
}

__global__ void hy_fill_kernel(uint32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__device__ inline int32_t hy_round(float x) {
    int32_t r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// The Hybrid Gridding Step for the chunks of a plan (see the file comment).
// A chunk's records (metadata and visibilities, gathered through the
// permutation with all loads in flight) are staged in LDS first, which also
// gives the chunk's bound; the waves then take every fourth record, four at
// a time, reading everything they need from LDS.
constexpr int kHyMaxR = 512;      // records per chunk (plan R is at most this)
constexpr int kHyUnroll = 4;

template <int NI>   // taps per lane: ceil(S / 8)
__global__ __launch_bounds__(kHyThreads) void hy_grid_kernel(
    HyGeom g, const uint2 *__restrict__ meta, const uint32_t *__restrict__ perm,
    const float *__restrict__ taps, const float *__restrict__ tmaxp,
    const Chunk *__restrict__ chunks, const int64_t *__restrict__ counters,
    const float *__restrict__ vis, float *__restrict__ grid) {
    // LDS: staged metadata [R], visibilities [R][8], tap table [beta S],
    // then the fixed-point region [kHyTV][RW][8]
    extern __shared__ int32_t lds[];
    uint2 *st_meta = reinterpret_cast<uint2 *>(lds);
    float *st_vis = reinterpret_cast<float *>(lds + 2 * kHyMaxR);
    float *st_tab = st_vis + 8 * kHyMaxR;
    const int S = g.S, npol = g.npol;
    const int ntab = (g.beta * S + 3) & ~3;
    int32_t *region = reinterpret_cast<int32_t *>(st_tab + ntab);
    __shared__ float s_part[kHyWaves];
    __shared__ int s_bad[kHyWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = lane & 7;               // component: polarisation c / 2, part c % 2
    const int i0 = lane >> 3;             // tap of the lane (plus multiples of 8)
    const int RW = kHyTU + S - 1;
    const bool comp_on = c < 2 * npol;
    const float tmax = *tmaxp;
    __shared__ int s_box[kHyWaves][4];
    for (int k = threadIdx.x; k < g.beta * S; k += kHyThreads) st_tab[k] = taps[k];
    const uint32_t nchunks = (uint32_t)counters[2];
    constexpr int kPer = kHyMaxR / kHyThreads;
    // the permutation entries and metadata of a chunk's records are loaded
    // one chunk ahead (they arrive while the previous chunk is gridded)
    uint32_t src[kPer];
    uint2 mrec[kPer];
    auto prefetch = [&](uint32_t cj) {
        Chunk cn{0u, 0u, 0u, 0u};
        if (cj < nchunks) cn = chunks[cj];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int j = threadIdx.x + k * kHyThreads;
            const bool on = j < (int)cn.len;
            src[k] = on ? perm[cn.start + j] : 0u;
            mrec[k] = on ? meta[cn.start + j] : make_uint2(0u, 0u);
        }
    };
    prefetch(blockIdx.x);
    for (uint32_t ci = blockIdx.x; ci < nchunks; ci += gridDim.x) {
        const Chunk ch = chunks[ci];
        const int tu0 = (int)(ch.bucket % (uint32_t)g.ntu) * kHyTU;
        const int tv0 = (int)(ch.bucket / (uint32_t)g.ntu) * kHyTV;
        const int len = (int)ch.len;
        // stage the chunk's visibilities (all loads in flight), its bound and
        // the bounding box of its footprints
        float part = 0.0f;
        bool bad = false;
        int rmin = kHyTV, rmax = -1, cmin = kHyTU, cmax = -1;
        float4 va[kPer], vb[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int j = threadIdx.x + k * kHyThreads;
            va[k] = vb[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (j >= len) continue;
            const float *v = vis + (size_t)src[k] * 2 * npol;
            if (npol == 4) {
                va[k] = reinterpret_cast<const float4 *>(v)[0];
                vb[k] = reinterpret_cast<const float4 *>(v)[1];
            } else {
                float xs[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) xs[q] = (q < 2 * npol) ? v[q] : 0.0f;
                va[k] = make_float4(xs[0], xs[1], xs[2], xs[3]);
                vb[k] = make_float4(xs[4], xs[5], xs[6], xs[7]);
            }
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int j = threadIdx.x + k * kHyThreads;
            if (j >= len) continue;
            st_meta[j] = mrec[k];
            const int row = (int)mrec[k].y - tv0, col = (int)(mrec[k].x & 0xffffu) - tu0;
            rmin = min(rmin, row);
            rmax = max(rmax, row);
            cmin = min(cmin, col);
            cmax = max(cmax, col);
            const float xs[8] = {va[k].x, va[k].y, va[k].z, va[k].w,
                                 vb[k].x, vb[k].y, vb[k].z, vb[k].w};
            float m = 0.0f;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                bad = bad || !isfinite(xs[q]);
                m = fmaxf(m, fabsf(xs[q]));
            }
            part += m;
        }
        prefetch(ci + gridDim.x);
        for (int off = 32; off > 0; off >>= 1) {
            part += __shfl_xor(part, off);
            rmin = min(rmin, __shfl_xor(rmin, off));
            rmax = max(rmax, __shfl_xor(rmax, off));
            cmin = min(cmin, __shfl_xor(cmin, off));
            cmax = max(cmax, __shfl_xor(cmax, off));
        }
        const bool wbad = __any(bad);
        if (lane == 0) {
            s_part[wave] = part;
            s_bad[wave] = wbad ? 1 : 0;
            s_box[wave][0] = rmin;
            s_box[wave][1] = rmax;
            s_box[wave][2] = cmin;
            s_box[wave][3] = cmax;
        }
        __syncthreads();
        float bound = 0.0f;
        int anybad = 0;
        rmin = kHyTV, rmax = -1, cmin = kHyTU, cmax = -1;
        for (int w = 0; w < kHyWaves; ++w) {
            bound += s_part[w];
            anybad |= s_bad[w];
            rmin = min(rmin, s_box[w][0]);
            rmax = max(rmax, s_box[w][1]);
            cmin = min(cmin, s_box[w][2]);
            cmax = max(cmax, s_box[w][3]);
        }
        // the touched part of the region: rows rmin..rmax, columns
        // cmin..cmax + S - 1 (a chunk has at least one record)
        const int bw = cmax + S - cmin, bh = rmax - rmin + 1;
        bound = 2.0f * tmax * bound * 1.0001f + 1e-30f;
        const bool use_lds = !anybad && isfinite(bound);
        int scale = 0;
        if (use_lds) {
            int e = 0;
            frexpf(bound, &e);
            scale = max(-120, min(120, 30 - e));
            for (int k = threadIdx.x; k < bh * bw * 8; k += kHyThreads) {
                const int cell = k >> 3, r = cell / bw, cc = cell - r * bw;
                region[((rmin + r) * RW + cmin + cc) * 8 + (k & 7)] = 0;
            }
        }
        // the staged visibilities carry the chunk's scale (exact powers of
        // two), so the accumulators are in units of the quantum
        {
            const float fs = ldexpf(1.0f, scale);
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int j = threadIdx.x + k * kHyThreads;
                if (j >= len) continue;
                reinterpret_cast<float4 *>(st_vis)[2 * j] =
                    make_float4(va[k].x * fs, va[k].y * fs, va[k].z * fs, va[k].w * fs);
                reinterpret_cast<float4 *>(st_vis)[2 * j + 1] =
                    make_float4(vb[k].x * fs, vb[k].y * fs, vb[k].z * fs, vb[k].w * fs);
            }
        }
        __syncthreads();

        // the waves take every fourth record, kHyUnroll at a time; lane
        // (tap i0 + 8 t, component c) adds one word per record
        auto records = [&](auto fixed_t) {
            constexpr bool FIXED = decltype(fixed_t)::value;
            for (int j0 = wave; j0 < len; j0 += kHyWaves * kHyUnroll) {
                uint32_t mx[kHyUnroll], mq[kHyUnroll];
                float x[kHyUnroll];
#pragma unroll
                for (int u = 0; u < kHyUnroll; ++u) {
                    const int j = min(j0 + u * kHyWaves, len - 1);
                    const uint2 m = st_meta[j];
                    mx[u] = uniform_u32(m.x);
                    mq[u] = uniform_u32(m.y);
                    x[u] = st_vis[8 * j + c];
                }
#pragma unroll
                for (int u = 0; u < kHyUnroll; ++u) {
                    if (j0 + u * kHyWaves >= len) break;
                    const int ku = (int)(mx[u] & 0xffffu), ou = (int)(mx[u] >> 16);
                    const int q = (int)mq[u];
#pragma unroll
                    for (int t = 0; t < NI; ++t) {
                        const int i = i0 + 8 * t;
                        if (i >= S) continue;
                        const float val = st_tab[ou * S + i] * x[u];
                        if (!comp_on) continue;
                        if constexpr (FIXED) {
                            atomicAdd(&region[((q - tv0) * RW + (ku - tu0) + i) * 8 + c],
                                      hy_round(val));
                        } else {
                            float *dst = grid + ((((size_t)(c >> 1) * g.rows + q) * g.nu + ku + i) *
                                                     2 + (c & 1));
                            unsafeAtomicAdd(dst, val);
                        }
                    }
                }
            }
        };
        if (use_lds)
            records(std::true_type{});
        else
            records(std::false_type{});
        __syncthreads();
        if (use_lds) {
            // polarisation by polarisation over the touched box, consecutive
            // threads on consecutive words of a grid row (re, im of
            // consecutive cells)
            const int per_pol = bh * bw * 2;
            for (int pol = 0; pol < npol; ++pol) {
                for (int k = threadIdx.x; k < per_pol; k += kHyThreads) {
                    const int part = k & 1, bc = k >> 1;
                    const int r = bc / bw;
                    const int row = rmin + r, col = cmin + (bc - r * bw);
                    const int32_t qv = region[(row * RW + col) * 8 + 2 * pol + part];
                    if (qv == 0 || tv0 + row >= g.rows || tu0 + col >= g.nu) continue;
                    float *dst = grid + ((((size_t)pol * g.rows + tv0 + row) * g.nu + tu0 + col) *
                                             2 + part);
                    unsafeAtomicAdd(dst, ldexpf((float)qv, -scale));
                }
            }
        }
        __syncthreads();
    }
}

// Column pruner: out[pol][j][col] = sum_{s, a} c(alpha (s - SZ/2) + a)
// in[pol][(alpha (j - SZ/2 + s) + a) mod M][col], c(d) = ztab[d + alpha SZ/2].
// A thread takes one column and J consecutive outputs; input block b (rows
// alpha b .. alpha b + alpha - 1) feeds outputs b - SZ/2 + 1 .. b + SZ/2;
// output j lives in ring slot (j - j0 + SZ - 1) mod SZ, which makes every
// slot index a compile-time constant of the unrolled loop, and is complete
// (written and cleared) once block j + SZ/2 - 1 has been added.
template <int SZ>
__global__ __launch_bounds__(256) void prune_columns_kernel(const float2 *__restrict__ in,
                                                            float2 *__restrict__ out,
                                                            int64_t M, int32_t ncols,
                                                            int32_t alpha, int32_t J,
                                                            const float *__restrict__ ztab) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int pol = blockIdx.z;
    const int64_t Mb = M / alpha;                      // output rows
    const int64_t j0 = (int64_t)blockIdx.y * J;
    const int64_t j_end = min<int64_t>(j0 + J, Mb);
    if (col >= ncols || j0 >= Mb) return;
    const float2 *src = in + (size_t)pol * M * ncols + col;
    float2 *dst = out + (size_t)pol * Mb * ncols + col;
    const int half = alpha * SZ / 2;
    float2 acc[SZ];
#pragma unroll
    for (int k = 0; k < SZ; ++k) acc[k] = make_float2(0.0f, 0.0f);
    const int64_t b0 = j0 - SZ / 2;
    const int64_t b1 = j_end - 1 + SZ / 2;             // last block
    for (int64_t bb = b0; bb <= b1; bb += SZ) {
#pragma unroll
        for (int t = 0; t < SZ; ++t) {
            const int64_t b = bb + t;
            if (b > b1) break;
            int64_t bw = b % Mb;                       // circular convolution
            if (bw < 0) bw += Mb;
            const float2 *row = src + (size_t)(bw * alpha) * ncols;
            for (int a = 0; a < alpha; ++a) {
                const float2 x = row[(size_t)a * ncols];
                // block b feeds output j = b + SZ/2 - s with coefficient
                // c(alpha (s - SZ/2) + a), slot (t - s - 1) mod SZ
#pragma unroll
                for (int s = 0; s < SZ; ++s) {
                    const float w = ztab[alpha * (s - SZ / 2) + a + half];
                    float2 &y = acc[((t - s - 1) % SZ + SZ) % SZ];
                    y.x = fmaf(w, x.x, y.x);
                    y.y = fmaf(w, x.y, y.y);
                }
            }
            const int64_t jc = b - SZ / 2 + 1;         // complete output
            if (jc >= j0 && jc < j_end) dst[(size_t)jc * ncols] = acc[t];
            acc[t] = make_float2(0.0f, 0.0f);
        }
    }
}

// The same map for a compile-time alpha.  A thread's J = 5 SZ + 1 outputs
// need exactly 6 SZ input blocks, so the unrolled block loop has no exit
// test and every block's alpha row loads are independent of the previous
// block's multiply-adds (the loads run ahead); blocks past the thread's last
// output wrap around the grid like the others and are never stored.  The
// block index advances with a wrap instead of a division.
template <int SZ, int ALPHA>
__global__ __launch_bounds__(256) void prune_columns_fixed_kernel(const float2 *__restrict__ in,
                                                                  float2 *__restrict__ out,
                                                                  int64_t M, int32_t ncols,
                                                                  const float *__restrict__ ztab) {
    constexpr int J = 5 * SZ + 1;
    constexpr int HALF = ALPHA * SZ / 2;
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int pol = blockIdx.z;
    const int64_t Mb = M / ALPHA;                      // output rows
    const int64_t j0 = (int64_t)blockIdx.y * J;
    const int64_t j_end = min<int64_t>(j0 + J, Mb);
    if (col >= ncols || j0 >= Mb) return;
    const float2 *src = in + (size_t)pol * M * ncols + col;
    float2 *dst = out + (size_t)pol * Mb * ncols + col;
    float2 acc[SZ];
#pragma unroll
    for (int k = 0; k < SZ; ++k) acc[k] = make_float2(0.0f, 0.0f);
    int64_t b = j0 - SZ / 2;
    int64_t bw = b % Mb;                               // circular convolution
    if (bw < 0) bw += Mb;
    for (int it = 0; it < 6; ++it) {
#pragma unroll
        for (int t = 0; t < SZ; ++t) {
            const float2 *row = src + (size_t)(bw * ALPHA) * ncols;
            float2 x[ALPHA];
#pragma unroll
            for (int a = 0; a < ALPHA; ++a) x[a] = row[(size_t)a * ncols];
#pragma unroll
            for (int a = 0; a < ALPHA; ++a) {
#pragma unroll
                for (int s = 0; s < SZ; ++s) {
                    const float w = ztab[ALPHA * (s - SZ / 2) + a + HALF];
                    float2 &y = acc[((t - s - 1) % SZ + SZ) % SZ];
                    y.x = fmaf(w, x[a].x, y.x);
                    y.y = fmaf(w, x[a].y, y.y);
                }
            }
            const int64_t jc = b - SZ / 2 + 1;         // complete output
            if (jc >= j0 && jc < j_end) dst[(size_t)jc * ncols] = acc[t];
            acc[t] = make_float2(0.0f, 0.0f);
            ++b;
            bw = (bw + 1 == Mb) ? 0 : bw + 1;
        }
    }
}

template <int SZ>
void launch_prune(const float2 *in, float2 *out, int npol, int64_t M, int ncols, int alpha,
                  const float *ztab, hipStream_t stream) {
    const int64_t Mb = M / alpha;
    if (alpha == 2 || alpha == 4 || alpha == 8) {
        constexpr int J = 5 * SZ + 1;
        const dim3 grid((unsigned)((ncols + 255) / 256), (unsigned)((Mb + J - 1) / J),
                        (unsigned)npol);
        if (alpha == 2)
            hipLaunchKernelGGL((prune_columns_fixed_kernel<SZ, 2>), grid, dim3(256), 0, stream,
                               in, out, M, ncols, ztab);
        else if (alpha == 4)
            hipLaunchKernelGGL((prune_columns_fixed_kernel<SZ, 4>), grid, dim3(256), 0, stream,
                               in, out, M, ncols, ztab);
        else
            hipLaunchKernelGGL((prune_columns_fixed_kernel<SZ, 8>), grid, dim3(256), 0, stream,
                               in, out, M, ncols, ztab);
        return;
    }
    constexpr int J = 64;
    const dim3 grid((unsigned)((ncols + 255) / 256), (unsigned)((Mb + J - 1) / J),
                    (unsigned)npol);
    hipLaunchKernelGGL(prune_columns_kernel<SZ>, grid, dim3(256), 0, stream, in, out, M, ncols,
                       alpha, J, ztab);
}

int grid_blocks_hy(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (int)std::max<int64_t>(1, std::min<int64_t>(8192, b));
}

}  // namespace
}  // namespace mg

struct mg_hybrid_plan {
    mg::HyGeom g{};
    mg_dtype tap_dtype = MG_F32;
    int64_t nrec = 0, nb = 0, max_chunks = 0;
    uint32_t R = 1024;
    // arena arrays
    float *taps = nullptr;
    float *tmax = nullptr;
    uint2 *meta = nullptr;
    uint32_t *perm = nullptr;
    mg::Chunk *chunks = nullptr;
    uint32_t *hist = nullptr, *bstart = nullptr, *cursor = nullptr, *cstart = nullptr;
    int64_t *counters = nullptr;
    size_t bytes = 0;
    void *owned = nullptr;
    hipStream_t create_stream = nullptr;
};

namespace mg {
namespace {

mg_status hy_check(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec, const void *uvw,
                   mg_dtype uvw_dtype) {
    if (!g || !k) return set_error(MG_EINVAL, "null descriptor");
    if (k->kind != MG_KERNEL_SEPARABLE)
        return set_error(MG_EINVAL, "hybrid gridding takes a separable kernel");
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
    if (k->support < 1 || k->support > kHyMaxS)
        return set_error(MG_EINVAL, "hybrid support must be in 1..32");
    if (((int64_t)g->beta * k->support) % 2) return set_error(MG_EINVAL, "beta * support must be even");
    if (k->ntaps < (int64_t)g->beta * k->support + 1)
        return set_error(MG_EINVAL, "separable table shorter than beta*S+1");
    return MG_OK;
}

void hy_prepare(mg_hybrid_plan &P, const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec) {
    P.g.nu = g->nu;
    P.g.nv = g->nv;
    P.g.npol = g->npol;
    P.g.beta = g->beta;
    P.g.S = k->support;
    P.g.rows = g->beta * g->nv;
    P.g.ntu = (g->nu + kHyTU - 1) / kHyTU;
    P.g.ntv = (P.g.rows + kHyTV - 1) / kHyTV;
    P.g.scale_u = g->scale_u;
    P.g.scale_v = g->scale_v;
    P.tap_dtype = k->tap_dtype;
    P.nrec = nrec;
    P.nb = (int64_t)P.g.ntu * P.g.ntv;
    P.R = (uint32_t)std::max<int64_t>(64, std::min<int64_t>(kHyMaxR, nrec / 4096));
    P.max_chunks = P.nb + nrec / P.R + 1;
}

template <typename F>
size_t hy_walk(const mg_hybrid_plan &P, F &&place) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += arena_round(bytes);
        return at;
    };
    const size_t n = (size_t)P.nrec + kRecPad;
    place(0, take(sizeof(float) * (size_t)P.g.beta * P.g.S));
    place(1, take(sizeof(float)));
    place(2, take(sizeof(uint2) * n));
    place(3, take(sizeof(uint32_t) * n));
    place(4, take(sizeof(Chunk) * (size_t)P.max_chunks));
    place(5, take(sizeof(uint32_t) * (size_t)P.nb));
    place(6, take(sizeof(uint32_t) * (size_t)P.nb));
    place(7, take(sizeof(uint32_t) * (size_t)P.nb));
    place(8, take(sizeof(uint32_t) * (size_t)(P.nb + 1)));
    place(9, take(sizeof(int64_t) * 4));
    return off;
}

void hy_carve(mg_hybrid_plan &P, void *arena) {
    char *base = static_cast<char *>(arena);
    P.bytes = hy_walk(P, [&](int what, size_t at) {
        void *p = base + at;
        switch (what) {
        case 0: P.taps = static_cast<float *>(p); break;
        case 1: P.tmax = static_cast<float *>(p); break;
        case 2: P.meta = static_cast<uint2 *>(p); break;
        case 3: P.perm = static_cast<uint32_t *>(p); break;
        case 4: P.chunks = static_cast<Chunk *>(p); break;
        case 5: P.hist = static_cast<uint32_t *>(p); break;
        case 6: P.bstart = static_cast<uint32_t *>(p); break;
        case 7: P.cursor = static_cast<uint32_t *>(p); break;
        case 8: P.cstart = static_cast<uint32_t *>(p); break;
        default: P.counters = static_cast<int64_t *>(p); break;
        }
    });
}

mg_status hy_build(mg_hybrid_plan &P, const mg_kernel_desc *k, const void *uvw, mg_dtype dt,
                   hipStream_t stream) {
    hipLaunchKernelGGL(hy_fill_kernel, dim3(1), dim3(64), 0, stream,
                       reinterpret_cast<uint32_t *>(P.counters), (int64_t)8);
    hipLaunchKernelGGL(hy_fill_kernel, dim3(1), dim3(64), 0, stream,
                       reinterpret_cast<uint32_t *>(P.tmax), (int64_t)1);
    hipLaunchKernelGGL(hy_fill_kernel, dim3(grid_blocks_hy(P.nb)), dim3(256), 0, stream, P.hist,
                       P.nb);
    if (P.tap_dtype == MG_F16)
        hipLaunchKernelGGL(hy_taps_kernel<__half>, dim3(1), dim3(256), 0, stream, P.g.beta, P.g.S,
                           (const __half *)k->taps, P.taps, P.tmax);
    else if (P.tap_dtype == MG_BF16)
        hipLaunchKernelGGL(hy_taps_kernel<__hip_bfloat16>, dim3(1), dim3(256), 0, stream, P.g.beta,
                           P.g.S, (const __hip_bfloat16 *)k->taps, P.taps, P.tmax);
    else
        hipLaunchKernelGGL(hy_taps_kernel<float>, dim3(1), dim3(256), 0, stream, P.g.beta, P.g.S,
                           (const float *)k->taps, P.taps, P.tmax);
    const int gb = grid_blocks_hy(P.nrec);
    if (P.nrec > 0) {
        if (dt == MG_F32)
            hipLaunchKernelGGL(hy_count_kernel<float>, dim3(gb), dim3(256), 0, stream, P.g, P.nrec,
                               (const float *)uvw, P.hist, P.counters);
        else
            hipLaunchKernelGGL(hy_count_kernel<double>, dim3(gb), dim3(256), 0, stream, P.g, P.nrec,
                               (const double *)uvw, P.hist, P.counters);
    }
    hipLaunchKernelGGL(hy_scan_kernel, dim3(1), dim3(256), 0, stream, P.hist, P.nb, P.R, P.bstart,
                       P.cursor, P.cstart, P.counters);
    if (P.nrec > 0) {
        if (dt == MG_F32)
            hipLaunchKernelGGL(hy_scatter_kernel<float>, dim3(gb), dim3(256), 0, stream, P.g,
                               P.nrec, (const float *)uvw, P.cursor, P.meta, P.perm);
        else
            hipLaunchKernelGGL(hy_scatter_kernel<double>, dim3(gb), dim3(256), 0, stream, P.g,
                               P.nrec, (const double *)uvw, P.cursor, P.meta, P.perm);
    }
    hipLaunchKernelGGL(hy_chunks_kernel, dim3(grid_blocks_hy(P.nb)), dim3(256), 0, stream, P.nb,
                       P.R, P.hist, P.bstart, P.cstart, P.chunks);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(MG_EDEVICE, std::string("hybrid plan kernels: ") + hipGetErrorString(e));
    return MG_OK;
}

mg_status hy_grid(const mg_hybrid_plan &P, const void *vis, void *grid, hipStream_t stream) {
    if (P.nrec == 0) return MG_OK;
    const size_t lds = sizeof(int32_t) * (size_t)(2 * kHyMaxR + 8 * kHyMaxR +
                                                  ((P.g.beta * P.g.S + 3) & ~3) +
                                                  kHyTV * (kHyTU + P.g.S - 1) * 8);
    auto launch = [&](auto kern) {
        const int groups = resident_groups((const void *)kern, kHyThreads, lds);
        hipLaunchKernelGGL(kern, dim3(groups), dim3(kHyThreads), lds, stream, P.g, P.meta,
                           P.perm, P.taps, P.tmax, P.chunks, P.counters, (const float *)vis,
                           (float *)grid);
    };
    const int ni = (P.g.S + 7) / 8;
    if (ni == 1) launch(hy_grid_kernel<1>);
    else if (ni == 2) launch(hy_grid_kernel<2>);
    else if (ni == 3) launch(hy_grid_kernel<3>);
    else launch(hy_grid_kernel<4>);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(MG_EDEVICE, std::string("hybrid grid kernel: ") + hipGetErrorString(e));
    return MG_OK;
}

__global__ void hy_add_count_kernel(const int64_t *src, int64_t *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst += *src;
}

}  // namespace
}  // namespace mg

using namespace mg;

extern "C" {

mg_status mg_hybrid_plan_workspace_size(const mg_grid_desc *g, const mg_kernel_desc *k,
                                        int64_t nrec, size_t *bytes) {
    if (!bytes) return set_error(MG_EINVAL, "null bytes output");
    *bytes = 0;
    mg_status s = hy_check(g, k, nrec, reinterpret_cast<const void *>(1), MG_F32);
    if (s != MG_OK) return s;
    mg_hybrid_plan P;
    hy_prepare(P, g, k, nrec);
    *bytes = hy_walk(P, [](int, size_t) {});
    return MG_OK;
}

mg_status mg_hybrid_plan_create(mg_hybrid_plan **plan, const mg_grid_desc *g,
                                const mg_kernel_desc *k, int64_t nrec, const void *uvw,
                                mg_dtype uvw_dtype, void *workspace, hipStream_t stream) {
    if (!plan) return set_error(MG_EINVAL, "null plan output");
    *plan = nullptr;
    mg_status s = hy_check(g, k, nrec, uvw, uvw_dtype);
    if (s != MG_OK) return s;
    if (workspace && (reinterpret_cast<uintptr_t>(workspace) % kArenaAlign) != 0)
        return set_error(MG_EINVAL, "workspace must be 256-byte aligned");
    mg_hybrid_plan *p = new (std::nothrow) mg_hybrid_plan;
    if (!p) return set_error(MG_ENOMEM, "host allocation failed");
    hy_prepare(*p, g, k, nrec);
    p->create_stream = stream;
    void *arena = workspace;
    if (!arena) {
        const size_t bytes = hy_walk(*p, [](int, size_t) {});
        const hipError_t e = scratch_alloc(&arena, bytes, stream);
        if (e != hipSuccess) {
            delete p;
            return set_error(MG_ENOMEM, std::string("hybrid plan allocation: ") + hipGetErrorString(e));
        }
        p->owned = arena;
    }
    hy_carve(*p, arena);
    s = hy_build(*p, k, uvw, uvw_dtype, stream);
    if (s != MG_OK) {
        if (p->owned) scratch_free(p->owned, stream);
        delete p;
        return s;
    }
    *plan = p;
    return MG_OK;
}

mg_status mg_hybrid_plan_grid(const mg_hybrid_plan *plan, const void *vis, void *grid,
                              hipStream_t stream) {
    if (!plan) return set_error(MG_EINVAL, "null plan");
    if (plan->nrec > 0 && !vis) return set_error(MG_EINVAL, "null vis");
    if (!grid) return set_error(MG_EINVAL, "null grid");
    return hy_grid(*plan, vis, grid, stream);
}

mg_status mg_hybrid_plan_nskipped(const mg_hybrid_plan *plan, int64_t *nskipped) {
    if (!plan || !nskipped) return set_error(MG_EINVAL, "null argument");
    if (hipStreamSynchronize(plan->create_stream) != hipSuccess)
        return set_error(MG_EDEVICE, "stream sync failed");
    int64_t v = 0;
    if (hipMemcpy(&v, plan->counters, sizeof v, hipMemcpyDeviceToHost) != hipSuccess)
        return set_error(MG_EDEVICE, "counter copy failed");
    *nskipped = v;
    return MG_OK;
}

mg_status mg_hybrid_plan_destroy(mg_hybrid_plan *plan) {
    if (!plan) return MG_OK;
    // a library-owned arena is released on the creating stream: calls on
    // other streams must have been ordered before the destroy by the caller
    if (plan->owned) scratch_free(plan->owned, plan->create_stream);
    delete plan;
    return MG_OK;
}

mg_status mg_hybrid_grid(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec,
                         const void *uvw, mg_dtype uvw_dtype, const void *vis, void *grid,
                         int64_t *d_nskipped, hipStream_t stream) {
    mg_status s = hy_check(g, k, nrec, uvw, uvw_dtype);
    if (s != MG_OK) return s;
    if (nrec > 0 && !vis) return set_error(MG_EINVAL, "null vis");
    if (!grid) return set_error(MG_EINVAL, "null grid");
    mg_hybrid_plan P;
    hy_prepare(P, g, k, nrec);
    void *arena = nullptr;
    const hipError_t e = scratch_alloc(&arena, hy_walk(P, [](int, size_t) {}), stream);
    if (e != hipSuccess) return set_error(MG_ENOMEM, std::string("hybrid scratch: ") + hipGetErrorString(e));
    hy_carve(P, arena);
    s = hy_build(P, k, uvw, uvw_dtype, stream);
    if (s == MG_OK) s = hy_grid(P, vis, grid, stream);
    if (s == MG_OK && d_nskipped)
        hipLaunchKernelGGL(hy_add_count_kernel, dim3(1), dim3(64), 0, stream, P.counters, d_nskipped);
    scratch_free(arena, stream);
    return s;
}

mg_status mg_prune_columns(int32_t npol, int64_t nrows, int32_t ncols, int32_t alpha,
                           int32_t support_z, const float *ztaps, const void *in, void *out,
                           hipStream_t stream) {
    if (npol < 1 || npol > 4 || nrows < 1 || ncols < 1 || alpha < 1)
        return set_error(MG_EINVAL, "bad pruning geometry");
    if (nrows % alpha) return set_error(MG_EINVAL, "nrows must be a multiple of alpha");
    if (support_z < 2 || support_z > 16 || support_z % 2)
        return set_error(MG_EINVAL, "pruning support must be even, 2..16");
    if (nrows / alpha > 0x7fffffffLL) return set_error(MG_EINVAL, "too many output rows");
    if (!ztaps || !in || !out) return set_error(MG_EINVAL, "null pointer");
    const float2 *src = static_cast<const float2 *>(in);
    float2 *dst = static_cast<float2 *>(out);
    switch (support_z) {
    case 2: launch_prune<2>(src, dst, npol, nrows, ncols, alpha, ztaps, stream); break;
    case 4: launch_prune<4>(src, dst, npol, nrows, ncols, alpha, ztaps, stream); break;
    case 6: launch_prune<6>(src, dst, npol, nrows, ncols, alpha, ztaps, stream); break;
    case 8: launch_prune<8>(src, dst, npol, nrows, ncols, alpha, ztaps, stream); break;
    case 10: launch_prune<10>(src, dst, npol, nrows, ncols, alpha, ztaps, stream); break;
    case 12: launch_prune<12>(src, dst, npol, nrows, ncols, alpha, ztaps, stream); break;
    case 14: launch_prune<14>(src, dst, npol, nrows, ncols, alpha, ztaps, stream); break;
    default: launch_prune<16>(src, dst, npol, nrows, ncols, alpha, ztaps, stream); break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(MG_EDEVICE, std::string("column pruner: ") + hipGetErrorString(e));
    return MG_OK;
}

}  // extern "C"
