// Degridding (gather): vis_out[r] = sum_{i,j} conj(w_ij) G[k_lo + (i, j)], the
// adjoint of the gridding map.
//
// Supports above 32 (degrid_block_kernel): work unit a unit, the chunks of
// one tile over the planes of the launch's group.  The grid region the unit
// can touch (its tile plus the group's largest S - 1 halo) is cut into
// 8 x 8-cell blocks, one cell per lane; block b belongs to wave b mod NW and
// its 4 polarisations stay in registers for the whole unit, so the grid is
// read once per unit with coalesced loads.  Every wave walks all records of
// the unit's chunks (scalar loads).  Per record, a vector compare and a ballot give the wave's blocks
// that the footprint overlaps; each takes one tap load and 16 multiply-adds
// per lane into the record's partial sums.  Partial sums of B records are
// then reduced across the wave's lanes (a butterfly that halves the values
// each lane holds at every step) and across the waves through LDS, and one
// thread per (record, component) writes the result.  Supports up to 32 take
// degrid_taps_kernel (below).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace mg {

namespace {

struct DegridParams {
    int32_t npol, nu, nv, beta;
    int32_t p_lo, p_hi;
};

// Next chunk of this launch (one vector atomic per chunk and workgroup).
__device__ inline uint32_t next_chunk_dg(uint32_t *queue, uint32_t *slot) {
    __syncthreads();
    if (threadIdx.x == 0) *slot = atomicAdd(queue, 1u);
    __syncthreads();
    return uniform_u32(*slot);
}

// Reduce-scatter over the 64 lanes of a wave.  On entry every lane holds N
// partial values (N a power of two, 2..32); on exit v[0] of lane l holds the
// wave-wide sum of value index reduce_index<N>(l).  Each halving step pairs
// every lane with the lane that differs in one bit: a lane keeps the half of
// its values selected by that bit and adds the partner's copy of the same
// half.  The bits are taken in the order 32, 16 (the gfx950 half-wave and
// row swaps, which exchange two registers in one instruction), then 8, 2, 1
// (DPP row rotation and quad permutes), then 4 (a swizzle); steps beyond
// log2(N) only add the partner's value, so lanes differing in those bits end
// with the same sum.
__device__ constexpr int kReduceBits[6] = {32, 16, 8, 2, 1, 4};

__device__ inline float dpp_xor(float x, int o) {
    const int xi = __float_as_int(x);
    int r;
    if (o == 8)
        r = __builtin_amdgcn_update_dpp(0, xi, 0x128, 0xf, 0xf, false);   // row_ror:8
    else if (o == 2)
        r = __builtin_amdgcn_update_dpp(0, xi, 0x4e, 0xf, 0xf, false);    // quad_perm 2,3,0,1
    else
        r = __builtin_amdgcn_update_dpp(0, xi, 0xb1, 0xf, 0xf, false);    // quad_perm 1,0,3,2
    return __int_as_float(r);
}

template <int N, int S, int H>
__device__ inline void reduce_step(float (&v)[N], int lane) {
    constexpr int o = kReduceBits[S];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        if constexpr (o == 32 || o == 16) {
            const auto r = (o == 32)
                               ? __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]),
                                                                  __float_as_uint(v[i + H]), false, false)
                               : __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]),
                                                                  __float_as_uint(v[i + H]), false, false);
            v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
        } else {
            const bool up = (lane & o) != 0;
            const float keep = up ? v[i + H] : v[i];
            const float send = up ? v[i] : v[i + H];
            v[i] = keep + dpp_xor(send, o);
        }
    }
    if constexpr (H > 1) reduce_step<N, S + 1, H / 2>(v, lane);
}

template <int N>
__device__ inline void wave_reduce_scatter(float (&v)[N], int lane) {
    static_assert(N >= 2 && N <= 32 && (N & (N - 1)) == 0, "N: power of two in [2, 32]");
    reduce_step<N, 0, N / 2>(v, lane);
    constexpr int kSteps = __builtin_ctz(N);
#pragma unroll
    for (int s = kSteps; s < 6; ++s) {
        const int o = kReduceBits[s];
        v[0] += (o == 4 || o == 32 || o == 16) ? __shfl_xor(v[0], o) : dpp_xor(v[0], o);
    }
}

// Value index held by `lane` after wave_reduce_scatter<N>.
template <int N>
__device__ inline int reduce_index(int lane) {
    constexpr int kSteps = __builtin_ctz(N);
    int idx = 0;
#pragma unroll
    for (int s = 0; s < kSteps; ++s) idx = 2 * idx + ((lane & kReduceBits[s]) ? 1 : 0);
    return idx;
}

// One lane per value index writes it: the lanes whose non-halving bits are 0.
template <int N>
__device__ inline bool reduce_writer(int lane) {
    constexpr int kSteps = __builtin_ctz(N);
    int mask = 0;
#pragma unroll
    for (int s = kSteps; s < 6; ++s) mask |= kReduceBits[s];
    return (lane & mask) == 0;
}

template <int KMAX, int NW, int B, bool SEP, typename TapT>
__global__ __launch_bounds__(NW * kWave) void degrid_block_kernel(
    const RecMeta *__restrict__ smeta, const uint32_t *__restrict__ sperm,
    const float *__restrict__ grid, float *__restrict__ vis_out, const TapT *__restrict__ taps,
    const Chunk *__restrict__ chunks, const uint32_t *__restrict__ bucket_cfirst,
    const uint2 *__restrict__ units, const uint32_t *__restrict__ group_nunits,
    const PlaneLayout *__restrict__ planes, uint32_t *__restrict__ queue, DegridParams prm) {
    constexpr int NV = B * 8;   // partial values per lane: B records x 4 pol x (re, im)
    constexpr uint32_t kElem = SEP ? sizeof(TapT) : 2 * sizeof(TapT);
    __shared__ float s_part[2][NW][NV];
    __shared__ uint32_t s_next;
    const int wave = (int)uniform_u32(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int lu = lane & 7, lv = lane >> 3;
    const int npol = prm.npol;
    const char *tbase = reinterpret_cast<const char *>(taps);
    const int my_idx = reduce_index<NV>(lane);
    const bool writer = reduce_writer<NV>(lane);
    int parity = 0;

    // The launch covers one plane group; its work items are units (chunks of
    // one tile over the group's planes), whose grid values are loaded once
    // over the tile plus the group's largest halo.
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
    // this lane's cell of each block (packed u | v << 16, region-relative)
    uint32_t cuv[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int b = k * NW + wave;
        cuv[k] = (uint32_t)(((b % nbx) << 3) + lu) | ((uint32_t)(((b / nbx) << 3) + lv) << 16);
    }

    for (uint32_t it = next_chunk_dg(queue, &s_next); it < nunits;
         it = next_chunk_dg(queue, &s_next)) {
        const uint2 un = gunits[it];
        const uint32_t c0 = un.x, c1 = un.x + un.y;
        const uint32_t t = (chunks[c0].bucket - gbase) / gn;
        const int cu0 = (int)((t % ntu) << g0.log2T);
        const int cv0 = (int)((t / ntu) << g0.log2T);
        // this lane's grid values of each block
        float g[KMAX][8];
        bool bad = false;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int b = k * NW + wave;
            const int u = cu0 + (int)(cuv[k] & 0xffffu), v = cv0 + (int)(cuv[k] >> 16);
            const bool in_grid = b < nblocks && u < prm.nu && v < prm.nv;
#pragma unroll
            for (int pol = 0; pol < 4; ++pol) {
                float2 x = make_float2(0.0f, 0.0f);
                if (in_grid && pol < npol)
                    x = *reinterpret_cast<const float2 *>(
                        grid + 2 * (((int64_t)pol * prm.nv + v) * prm.nu + u));
                g[k][2 * pol] = x.x;
                g[k][2 * pol + 1] = x.y;
                bad = bad || !isfinite(x.x) || !isfinite(x.y);
            }
        }
        // a zero tap times a non-finite grid value is NaN: units whose region
        // holds one mask the taps outside each footprint instead
        const bool exact = __syncthreads_or(bad) != 0;

        for (uint32_t c = c0; c < c1; ++c) {
            const Chunk ch = chunks[c];
            const int S = planes[g0.grp_first + (int)((ch.bucket - gbase) % gn)].S;
            // this lane's tap offset in each block, in bytes relative to the
            // footprint's first tap
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

            auto visit = [&](const RecMeta m, float (&acc)[8], auto exact_t) {
                constexpr bool EXACT = decltype(exact_t)::value;
                const uint32_t a = meta_ku(m) & (uint32_t)Tm;
                const uint32_t bq = meta_kv(m) & (uint32_t)Tm;
                const uint32_t hit = (uint32_t)__ballot((blo_u + 7u - a <= (uint32_t)(S + 6)) &&
                                                        (blo_v + 7u - bq <= (uint32_t)(S + 6)));
                const uint32_t full = (uint32_t)__ballot((blo_u - a <= (uint32_t)(S - 8)) &&
                                                         (blo_v - bq <= (uint32_t)(S - 8)));
                const uint32_t ab = a | (bq << 16);
                const char *tb;
                const char *tbv = nullptr;
                if constexpr (SEP) {
                    tb = tbase + ((int64_t)(m.toff & 0xffffu) - (int64_t)a) * (int64_t)kElem;
                    tbv = tbase + ((int64_t)(m.toff >> 16) - (int64_t)bq) * (int64_t)kElem;
                } else {
                    tb = tbase +
                         ((int64_t)m.toff - (int64_t)(bq * (uint32_t)S + a)) * (int64_t)kElem;
                }
                auto tap = [&](const int k) {
                    uint32_t o = voff[k];
                    asm volatile("" : "+v"(o));   // keeps the offset 32-bit: scalar-base load
                    if constexpr (SEP) {
                        uint32_t ov = voffv[k];
                        asm volatile("" : "+v"(ov));
                        const float t = TapTraits<TapT>::real((const TapT *)(tb + o), 0) *
                                        TapTraits<TapT>::real((const TapT *)(tbv + ov), 0);
                        return make_float2(t, 0.0f);
                    } else {
                        return TapTraits<TapT>::cplx((const TapT *)(tb + o), 0);
                    }
                };
                // acc += conj(w) * G = (wr gr + wi gi) + j (wr gi - wi gr)
                auto madd = [&](const int k, const float2 w) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float gr = g[k][2 * q], gi = g[k][2 * q + 1];
                        acc[2 * q] = fmaf(w.x, gr, fmaf(w.y, gi, acc[2 * q]));
                        acc[2 * q + 1] = fmaf(w.x, gi, fmaf(-w.y, gr, acc[2 * q + 1]));
                    }
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
                    float2 w[KMAX];
#pragma unroll
                    for (int k = 0; k < KMAX; ++k) {
                        w[k] = make_float2(0.0f, 0.0f);
                        if (!((hit >> k) & 1u)) continue;
                        const uint32_t d = cuv[k] - ab;
                        if (((full >> k) & 1u) || max(d & 0xffffu, d >> 16) < (uint32_t)S)
                            w[k] = tap(k);
                    }
#pragma unroll
                    for (int k = 0; k < KMAX; ++k)
                        if ((hit >> k) & 1u) madd(k, w[k]);
                }
            };

            auto records = [&](auto exact_t) {
                const uint32_t rend = ch.start + ch.len;
                // the next group's records are loaded while this group's taps are
                // (indices clamped into the chunk)
                RecMeta mnext[B];
                auto load_meta = [&](const uint32_t r) {
#pragma unroll
                    for (int bi = 0; bi < B; ++bi)
                        mnext[bi] = smeta[min(r + (uint32_t)bi, rend - 1)];
                };
                load_meta(ch.start);
                for (uint32_t r0 = ch.start; r0 < rend; r0 += B) {
                    const uint32_t nb = min((uint32_t)B, rend - r0);
                    // destination of the sums this thread writes (read now, used
                    // after the reductions)
                    const uint32_t dst = sperm[r0 + min((uint32_t)threadIdx.x >> 3, nb - 1)];
                    RecMeta m[B];
#pragma unroll
                    for (int bi = 0; bi < B; ++bi) m[bi] = mnext[bi];
                    load_meta(r0 + B);
                    float part[NV];
#pragma unroll
                    for (int i = 0; i < NV; ++i) part[i] = 0.0f;
#pragma unroll
                    for (int bi = 0; bi < B; ++bi) {
                        if ((uint32_t)bi < nb) {
                            float acc[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                            visit(m[bi], acc, exact_t);
#pragma unroll
                            for (int q = 0; q < 8; ++q) part[bi * 8 + q] = acc[q];
                        }
                    }
                    wave_reduce_scatter<NV>(part, lane);
                    if (writer) s_part[parity][wave][my_idx] = part[0];
                    __syncthreads();
                    if ((int)threadIdx.x < NV) {
                        const int bi = threadIdx.x >> 3, q = threadIdx.x & 7;
                        if ((uint32_t)bi < nb && (q >> 1) < npol) {
                            float sum = 0.0f;
#pragma unroll
                            for (int w = 0; w < NW; ++w) sum += s_part[parity][w][threadIdx.x];
                            vis_out[((size_t)dst * npol + (q >> 1)) * 2 + (q & 1)] = sum;
                        }
                    }
                    // the other buffer takes the next group, so one barrier per
                    // group keeps the readers ahead of the next writers
                    parity ^= 1;
                }
            };
            if (exact)
                records(std::true_type{});
            else
                records(std::false_type{});
        }
    }
}

// Supports up to 32: the lanes of a wave take the taps of one record (tap
// q = t * 64 + lane, q < S^2), so no lane sits outside a footprint.  A
// workgroup takes a unit (chunks of one tile over the planes of the group);
// the unit's grid region is staged once in LDS as [row][pol][col] float2
// rows of PITCH columns (a row stride of 4 PITCH + 8 float2, 16 banks
// modulo 64, spreads the rows of a footprint over the LDS banks); the
// waves of the workgroup take groups of B records in turn, and each group's
// sums are reduced across the wave's lanes only.
template <int PITCH>
constexpr int row_stride() { return 4 * PITCH + 8; }

// Waves per workgroup of the taps kernel: the S <= 8 and S <= 32 instances
// share each staged region among eight waves, which doubles the waves a CU
// holds where the region's LDS (S <= 32) or the workgroup count (S <= 8)
// limits them; the S <= 16 instance is held to four waves per SIMD by its
// registers either way.
constexpr int taps_waves(int ntap) { return ntap == 4 ? 4 : 8; }

template <int NTAP, int PITCH, int B, bool SEP, typename TapT>
__global__ __launch_bounds__(kWave * taps_waves(NTAP)) void degrid_taps_kernel(
    const RecMeta *__restrict__ smeta, const uint32_t *__restrict__ sperm,
    const float *__restrict__ grid, float *__restrict__ vis_out, const TapT *__restrict__ taps,
    const Chunk *__restrict__ chunks, const uint32_t *__restrict__ bucket_cfirst,
    const uint2 *__restrict__ units, const uint32_t *__restrict__ group_nunits,
    const PlaneLayout *__restrict__ planes, uint32_t *__restrict__ queue, DegridParams prm) {
    constexpr int NV = B * 8;
    constexpr int kWaves = taps_waves(NTAP);
    constexpr int kThreads = kWave * kWaves;
    constexpr uint32_t kElem = SEP ? sizeof(TapT) : 2 * sizeof(TapT);
    constexpr int kPitch = PITCH;
    constexpr int kRowStride = row_stride<PITCH>();
    extern __shared__ float2 region[];   // [row][pol][PITCH], row stride kRowStride
    __shared__ uint32_t s_next;
    const int wave = (int)uniform_u32(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int npol = prm.npol;
    const char *tbase = reinterpret_cast<const char *>(taps);
    const int my_idx = reduce_index<NV>(lane);
    const bool writer = reduce_writer<NV>(lane);
    // the launch covers one plane group; its work items are the group's
    // units (chunks of one tile over the group's planes), whose region is
    // staged once for all their chunks
    const PlaneLayout gl = planes[prm.p_lo];
    const uint2 *gunits = units + bucket_cfirst[gl.base];
    const uint32_t nunits = group_nunits[prm.p_lo];

    for (uint32_t it = next_chunk_dg(queue, &s_next); it < nunits;
         it = next_chunk_dg(queue, &s_next)) {
        const uint2 un = gunits[it];
        const uint32_t c0 = un.x, c1 = un.x + un.y;
        // region: union of the chunks' k_lo ranges extended by their supports
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
        const int cu0 = (int)(((tile % (uint32_t)gl.ntu) << gl.log2T) + umin);
        const int cv0 = (int)(((tile / (uint32_t)gl.ntu) << gl.log2T) + vmin);
        const int RW = (int)(uend - umin);
        const int RH = (int)(vend - vmin);

        // stage the region (cells outside it are never read); cell
        // j = rv * RW + ru of each polarisation, a thread stepping j by the
        // workgroup size and (rv, ru) by a fixed step (no division per cell)
        {
            const int cells = RH * RW;
            const int step_u = kThreads % RW, step_v = kThreads / RW;
            const int ru0 = (int)threadIdx.x % RW, rv0 = (int)threadIdx.x / RW;
            for (int pol = 0; pol < npol; ++pol) {
                const float2 *gp = reinterpret_cast<const float2 *>(grid) +
                                   ((int64_t)pol * prm.nv + cv0) * prm.nu + cu0;
                int ru = ru0, rv = rv0;
                for (int j = threadIdx.x; j < cells; j += kThreads) {
                    region[rv * kRowStride + pol * kPitch + ru] = gp[(int64_t)rv * prm.nu + ru];
                    ru += step_u;
                    rv += step_v;
                    if (ru >= RW) {
                        ru -= RW;
                        ++rv;
                    }
                }
            }
        }
        __syncthreads();

        uint32_t turn = 0;   // the wave whose turn it is, over the unit's groups
        for (uint32_t c = c0; c < c1; ++c) {
            const Chunk ch = chunks[c];
            int pc;
            uint32_t tile_;
            bucket_plane_tile(gl, ch.bucket, &pc, &tile_);
            const int S = planes[pc].S;

            // this lane's taps q = t * 64 + lane: LDS offset and table byte
            // offset relative to the footprint's first cell and first tap.
            // Taps t < nt - 1 lie in every footprint; where S^2 is not a
            // multiple of 64, lanes past S^2 in the last tap read the first
            // tap and first cell (in bounds) and their products are zeroed.
            const int nt_rt = (S * S + 63) >> 6;
            const bool last_full = (S * S) % 64 == 0;
            const bool last_on = ((nt_rt - 1) * 64 + lane) < S * S;
            // NT: taps held per lane; a compile-time count (one instance per
            // count) for up to 4 taps, else NTAP with the count tested
            auto run = [&](auto nt_t) {
                constexpr int NT = decltype(nt_t)::value;
                const int nt = (NTAP <= 4) ? NT : nt_rt;
                int lg[NT];
                uint32_t lt[NT], ltv[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int q = min(t * 64 + lane, S * S - 1);
                    const int qq = (t * 64 + lane < S * S) ? q : 0;
                    const int j = qq / S, i = qq - (qq / S) * S;
                    lg[t] = j * kRowStride + i;
                    if constexpr (SEP) {
                        lt[t] = (uint32_t)i * kElem;
                        ltv[t] = (uint32_t)j * kElem;
                    } else {
                        lt[t] = (uint32_t)(j * S + i) * kElem;
                        ltv[t] = 0u;
                    }
                }
                // the last tap's offsets (its index is a run-time value for
                // NTAP > 4: picked once per chunk)
                int lg_last = lg[0];
                uint32_t lt_last = lt[0], ltv_last = ltv[0];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    if (t == nt - 1) {
                        lg_last = lg[t];
                        lt_last = lt[t];
                        ltv_last = ltv[t];
                    }
                }

                // groups of B records, taken by the waves in turn (continuing
                // from the unit's previous chunk); a short last group repeats
                // the chunk's last record (its sums are not written)
                const uint32_t rend = ch.start + ch.len;
                const uint32_t ngroups = (ch.len + B - 1) / B;
                const uint32_t gfirst = ((uint32_t)wave + kWaves - turn) % kWaves;
                turn = (turn + ngroups) % kWaves;
                // the records of this wave's next group are loaded while the
                // current group's taps are (indices clamped into the chunk)
                RecMeta mnext[B];
                auto load_meta = [&](const uint32_t g) {
#pragma unroll
                    for (int bi = 0; bi < B; ++bi)
                        mnext[bi] = smeta[min(ch.start + g * B + (uint32_t)bi, rend - 1)];
                };
                load_meta(gfirst);
                for (uint32_t gi = gfirst; gi < ngroups; gi += kWaves) {
                    const uint32_t r0 = ch.start + gi * B;
                    const uint32_t nb = min((uint32_t)B, rend - r0);
                    // destination of this lane's sum (read now, used after the
                    // reduction)
                    const uint32_t dst = sperm[r0 + min((uint32_t)(my_idx >> 3), nb - 1)];
                    float part[NV];
#pragma unroll
                    for (int i = 0; i < NV; ++i) part[i] = 0.0f;
                    // record bi of the group: its LDS offset and tap pointers
                    int sg[B];
                    const char *tb[B];
                    const char *tbv[B];
#pragma unroll
                    for (int bi = 0; bi < B; ++bi) {
                        const RecMeta m = mnext[bi];
                        sg[bi] = ((int)meta_kv(m) - cv0) * kRowStride + ((int)meta_ku(m) - cu0);
                        if constexpr (SEP) {
                            tb[bi] = tbase + (size_t)(m.toff & 0xffffu) * kElem;
                            tbv[bi] = tbase + (size_t)(m.toff >> 16) * kElem;
                        } else {
                            tb[bi] = tbase + (size_t)m.toff * kElem;
                            tbv[bi] = nullptr;
                        }
                    }
                    load_meta(gi + kWaves);
                    // tap weight and the 4 grid values of one tap of record bi
                    auto load = [&](const int bi, const int g_off, uint32_t o, uint32_t ov,
                                    float2 &w, float2 (&gv)[4]) {
                        asm volatile("" : "+v"(o));   // keeps the offset 32-bit: scalar-base load
                        if constexpr (SEP) {
                            asm volatile("" : "+v"(ov));
                            w = make_float2(TapTraits<TapT>::real((const TapT *)(tb[bi] + o), 0) *
                                                TapTraits<TapT>::real((const TapT *)(tbv[bi] + ov), 0),
                                            0.0f);
                        } else {
                            w = TapTraits<TapT>::cplx((const TapT *)(tb[bi] + o), 0);
                        }
                        const float2 *gp = region + sg[bi] + g_off;
#pragma unroll
                        for (int q = 0; q < 4; ++q) gv[q] = gp[q * kPitch];
                    };
                    // lanes past S^2 in the last tap contribute nothing
                    auto mask_last = [&](float2 &w, float2 (&gv)[4]) {
                        if (!last_on) {
                            w = make_float2(0.0f, 0.0f);
#pragma unroll
                            for (int q = 0; q < 4; ++q) gv[q] = make_float2(0.0f, 0.0f);
                        }
                    };
                    // record bi's sums += conj(w) * G
                    auto fma4 = [&](const int bi, const float2 w, const float2 (&gv)[4]) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            float &ar = part[bi * 8 + 2 * q];
                            float &ai = part[bi * 8 + 2 * q + 1];
                            ar = fmaf(w.x, gv[q].x, fmaf(w.y, gv[q].y, ar));
                            ai = fmaf(w.x, gv[q].y, fmaf(-w.y, gv[q].x, ai));
                        }
                    };
                    if constexpr (NTAP > 4) {
#pragma unroll
                        for (int bi = 0; bi < B; ++bi) {
                            // many taps per lane: four at a time (their loads
                            // in flight together; the LDS region already
                            // limits the kernel to two waves per SIMD, so the
                            // registers are there)
#pragma unroll
                            for (int t = 0; t < NT - 1; t += 4) {
                                if (t < nt - 1) {
                                    float2 w[4], gv[4][4];
#pragma unroll
                                    for (int u = 0; u < 4; ++u)
                                        if (t + u < NT - 1 && t + u < nt - 1)
                                            load(bi, lg[t + u], lt[t + u], ltv[t + u], w[u], gv[u]);
#pragma unroll
                                    for (int u = 0; u < 4; ++u)
                                        if (t + u < NT - 1 && t + u < nt - 1) fma4(bi, w[u], gv[u]);
                                }
                            }
                            float2 w, gv[4];
                            load(bi, lg_last, lt_last, ltv_last, w, gv);
                            if (!last_full) mask_last(w, gv);
                            fma4(bi, w, gv);
                        }
                    } else {
                        // every tap of the group's records loaded, then the
                        // multiply-adds
                        float2 w[B][NT], gv[B][NT][4];
#pragma unroll
                        for (int bi = 0; bi < B; ++bi)
#pragma unroll
                            for (int t = 0; t < NT; ++t)
                                load(bi, lg[t], lt[t], ltv[t], w[bi][t], gv[bi][t]);
#pragma unroll
                        for (int bi = 0; bi < B; ++bi) {
                            if (!last_full) mask_last(w[bi][NT - 1], gv[bi][NT - 1]);
#pragma unroll
                            for (int t = 0; t < NT; ++t) fma4(bi, w[bi][t], gv[bi][t]);
                        }
                    }
                    wave_reduce_scatter<NV>(part, lane);
                    if (writer) {
                        const int bi = my_idx >> 3, q = my_idx & 7;
                        if ((uint32_t)bi < nb && (q >> 1) < npol)
                            vis_out[((size_t)dst * npol + (q >> 1)) * 2 + (q & 1)] = part[0];
                    }
                }
            };
            if constexpr (NTAP <= 4) {
                switch (nt_rt) {
                case 1: run(std::integral_constant<int, 1>{}); break;
                case 2: run(std::integral_constant<int, (NTAP < 2 ? NTAP : 2)>{}); break;
                case 3: run(std::integral_constant<int, (NTAP < 3 ? NTAP : 3)>{}); break;
                default: run(std::integral_constant<int, NTAP>{}); break;
                }
            } else {
                run(std::integral_constant<int, NTAP>{});
            }
        }
    }
}

// Outputs of skipped records are zero: they follow the valid ones in the
// plan's sorted order.
__global__ __launch_bounds__(256) void zero_skipped_kernel(const int64_t *__restrict__ counters,
                                                           int64_t nrec,
                                                           const uint32_t *__restrict__ sperm,
                                                           int32_t npol,
                                                           float2 *__restrict__ vis_out) {
    const int64_t nvalid = counters[1];
    for (int64_t i = nvalid + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrec;
         i += (int64_t)gridDim.x * blockDim.x) {
        float2 *o = vis_out + (size_t)sperm[i] * npol;
        for (int q = 0; q < npol; ++q) o[q] = make_float2(0.0f, 0.0f);
    }
}

__global__ void clear_queue_kernel(uint32_t *w, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) w[i] = 0u;
}

struct DegridPtrs {
    const RecMeta *smeta;
    const uint32_t *sperm;
    const float *grid;
    float *vis_out;
    const void *taps;
    const Chunk *chunks;
    const uint32_t *bucket_cfirst;
    const uint2 *units;
    const uint32_t *group_nunits;
    const PlaneLayout *planes;
    uint32_t *queue;
};

template <int KMAX, int NW, int B, bool SEP, typename TapT>
hipError_t launch_dg(const DegridPtrs &a, const DegridParams &prm, int tile, int smax,
                     hipStream_t stream) {
    // every block of the largest region has an owner
    const int side = (tile + smax - 1 + 7) / 8;
    if (side * side > KMAX * NW) return hipErrorInvalidValue;
    auto kern = degrid_block_kernel<KMAX, NW, B, SEP, TapT>;
    hipLaunchKernelGGL(kern, dim3(resident_groups((const void *)kern, NW * kWave, 0)),
                       dim3(NW * kWave), 0,
                       stream, a.smeta, a.sperm, a.grid, a.vis_out, (const TapT *)a.taps,
                       a.chunks, a.bucket_cfirst, a.units, a.group_nunits, a.planes, a.queue,
                       prm);
    return hipGetLastError();
}

template <int NTAP, int PITCH, bool SEP, typename TapT>
hipError_t launch_dt(const DegridPtrs &a, const DegridParams &prm, int tile, int smax,
                     hipStream_t stream) {
    // the region must fit the compile-time pitch and the taps the lanes
    if (tile + smax - 1 > PITCH || smax * smax > NTAP * 64) return hipErrorInvalidValue;
    const size_t lds = sizeof(float2) * (size_t)row_stride<PITCH>() * (size_t)(tile + smax - 1);
    // records per reduction group: two where a lane holds several taps
    // (registers; the reduction costs about the same per record either way)
    auto kern = degrid_taps_kernel<NTAP, PITCH, (NTAP > 1 ? 2 : 4), SEP, TapT>;
    constexpr int threads = kWave * taps_waves(NTAP);
    hipLaunchKernelGGL(kern, dim3(resident_groups((const void *)kern, threads, lds)),
                       dim3(threads), lds,
                       stream, a.smeta, a.sperm, a.grid, a.vis_out, (const TapT *)a.taps,
                       a.chunks, a.bucket_cfirst, a.units, a.group_nunits, a.planes, a.queue,
                       prm);
    return hipGetLastError();
}

template <bool SEP, typename TapT>
hipError_t launch_deg(int cls, const DegridPtrs &a, const DegridParams &prm, int tile, int smax,
                      hipStream_t stream) {
    switch (cls) {
    case 0: return launch_dt<1, 32, SEP, TapT>(a, prm, tile, smax, stream);
    case 1: return launch_dt<4, 32, SEP, TapT>(a, prm, tile, smax, stream);
    case 2: return launch_dt<16, 48, SEP, TapT>(a, prm, tile, smax, stream);
    default: return launch_dg<7, 16, 2, SEP, TapT>(a, prm, tile, smax, stream);
    }
}

template <bool SEP>
hipError_t launch_deg_t(mg_dtype dt, int cls, const DegridPtrs &a, const DegridParams &prm,
                        int tile, int smax, hipStream_t stream) {
    switch (dt) {
    case MG_F16: return launch_deg<SEP, __half>(cls, a, prm, tile, smax, stream);
    case MG_BF16: return launch_deg<SEP, __hip_bfloat16>(cls, a, prm, tile, smax, stream);
    default: return launch_deg<SEP, float>(cls, a, prm, tile, smax, stream);
    }
}

}  // namespace

size_t degrid_scratch_bytes(const PlanState &P) {
    return arena_round(sizeof(uint32_t) * (size_t)P.nplanes_eff);
}

mg_status launch_degrid(const PlanState &P, const void *grid, void *vis_out, void *scratch,
                        hipStream_t stream) {
    if (P.nrec == 0) return MG_OK;
    const int np = P.nplanes_eff;
    uint32_t *queues = static_cast<uint32_t *>(scratch);
    hipError_t e = hipSuccess;
    if (!queues) {
        e = scratch_alloc((void **)&queues, degrid_scratch_bytes(P), stream);
        if (e != hipSuccess) return set_error(MG_ENOMEM, "degrid: work queue allocation failed");
    }
    hipLaunchKernelGGL(clear_queue_kernel, dim3(1), dim3(256), 0, stream, queues, np);
    {
        int64_t nb = (P.nrec + 255) / 256;
        if (nb > 4096) nb = 4096;
        hipLaunchKernelGGL(zero_skipped_kernel, dim3((unsigned)nb), dim3(256), 0, stream,
                           P.counters, P.nrec, P.sperm, P.geom.npol, (float2 *)vis_out);
    }
    DegridPtrs a{P.smeta,    P.sperm,         (const float *)grid, (float *)vis_out,
                 P.taps,     P.chunks,        P.bucket_cfirst,     P.units,
                 P.group_nunits, P.d_planes,  nullptr};
    DegridParams prm{P.geom.npol, P.geom.nu, P.geom.nv, P.geom.beta, 0, 0};
    const bool sep = P.kind == MG_KERNEL_SEPARABLE;
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
        a.queue = queues + p0;
        const int cls = P.planes[p0].cls;
        e = sep ? launch_deg_t<true>(P.tap_dtype, cls, a, prm, P.planes[p0].T, smax, stream)
                : launch_deg_t<false>(P.tap_dtype, cls, a, prm, P.planes[p0].T, smax, stream);
        p0 = p1;
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (!scratch) scratch_free(queues, stream);
    if (e != hipSuccess) return set_error(MG_EDEVICE, std::string("degrid kernels: ") + hipGetErrorString(e));
    return MG_OK;
}

}  // namespace mg
