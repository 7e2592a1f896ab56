// Gridding (scatter) kernels.
//
// Work unit: one chunk = up to R records of one (plane, uv tile) bucket,
// cell-sorted.  A workgroup of 4 waves takes a chunk:
//
//  * Each wave keeps a moving window of grid cells in registers.  The
//    window has one slot per kernel tap offset class: slot (su, sv),
//    0 <= su, sv < S, owns the grid cells congruent to (su, sv) modulo S.
//    Every record's S x S footprint holds exactly one cell of each class,
//    so for every record every slot has work, and a slot's accumulators
//    (4 polarisations, complex) keep summing contributions while its cell
//    stays inside the footprint of consecutive records.  This is the
//    owner-computes scheme of Romein's GPU gridder, which the thesis's
//    Convolutional Gridder builds on (Chapter 4); here the slots are spread
//    over the 64 lanes of a wave (K slots per lane) and the records come
//    cell-sorted, so windows move rarely.
//  * When a slot's cell leaves the footprint its sums are committed into an
//    LDS copy of the chunk's grid region (tile plus S-1 halo), which all 4
//    waves share (LDS float atomics).  At the end of the chunk the region
//    is added to the grid in HBM with coalesced float atomics, so each grid
//    cell sees at most one HBM update per chunk.
//  * For supports above 32 the LDS region does not fit; the 4 waves split
//    the S^2 slots between them and commit straight to HBM.
//
// All polarisations are handled per visit: one tap load feeds 4 complex
// multiply-adds (the thesis's Polarisation Gain, Section 3.5).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mg {

namespace {

constexpr uint32_t kNoCell = 0xffffffffu;

struct GridParams {
    int32_t npol, nu, nv, beta;
    int32_t p_lo, p_hi;       // planes handled by this launch
};

// Records processed per batch of scalar loads (fewer for many slots per
// lane, to bound the registers holding the batch's taps).
template <int KMAX> struct BatchOf { static constexpr int value = KMAX >= 8 ? 2 : 4; };

// KMAX: slots per lane (compile-time upper bound); NG: slot groups (waves
// that share one chunk's records but own different slots); LDS: commit into
// the shared LDS region (else straight into the grid).
//
// Per record the wave does, on the scalar unit: decode the packed indices,
// fold the table conjugation into the visibilities, form the record's tap
// base.  Per slot, on the vector unit: one tap load (SGPR base + the slot's
// cached byte offset) and 16 FMAs (4 polarisations x complex).  The slot
// offsets and the window test are redone only when the record's first cell
// differs from the previous record's; records are cell-sorted, so runs of
// records share it.
template <int KMAX, int NG, bool SEP, typename TapT, bool LDS>
__global__ __launch_bounds__(kGroupThreads) void grid_window_kernel(
    const RecMeta *__restrict__ smeta, const float4 *__restrict__ svis, float *__restrict__ grid,
    const TapT *__restrict__ taps, const Chunk *__restrict__ chunks,
    const uint32_t *__restrict__ plane_cfirst, const PlaneLayout *__restrict__ planes,
    GridParams prm) {
    extern __shared__ float2 region[];
    constexpr int NSPLIT = kWavesPerGroup / NG;
    constexpr int kBatch = BatchOf<KMAX>::value;
    constexpr uint32_t kElem = SEP ? sizeof(TapT) : 2 * sizeof(TapT);   // bytes per tap
    const int wave = (int)uniform_u32(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int grp = wave % NG;
    const int split = wave / NG;
    const int npol = prm.npol;
    const int beta = prm.beta;
    const uint32_t c_begin = plane_cfirst[prm.p_lo];
    const uint32_t c_end = plane_cfirst[prm.p_hi];

    for (uint32_t c = c_begin + blockIdx.x; c < c_end; c += gridDim.x) {
        const Chunk ch = chunks[c];
        int p = prm.p_lo;
        while (p + 1 < prm.p_hi && (int64_t)ch.bucket >= planes[p + 1].base) ++p;
        const PlaneLayout pl = planes[p];
        const int S = pl.S;
        const uint32_t local = ch.bucket - (uint32_t)pl.base;
        const uint32_t tu0 = (local % (uint32_t)pl.ntu) << pl.log2T;
        const uint32_t tv0 = (local / (uint32_t)pl.ntu) << pl.log2T;
        const uint32_t cu0 = tu0 + (ch.bbox & 0xffu);
        const uint32_t cv0 = tv0 + ((ch.bbox >> 16) & 0xffu);
        const int RW = (int)((ch.bbox >> 8) & 0xffu) - (int)(ch.bbox & 0xffu) + S;
        const int RH = (int)(ch.bbox >> 24) - (int)((ch.bbox >> 16) & 0xffu) + S;
        const uint32_t rowlen = (uint32_t)pl.rowlen;
        const char *tplane = reinterpret_cast<const char *>(taps) + (size_t)pl.tap_off * kElem;

        if constexpr (LDS) {
            for (int i = threadIdx.x; i < npol * RH * RW; i += kGroupThreads)
                region[i] = make_float2(0.0f, 0.0f);
            __syncthreads();
        }

        // slots of this wave; invalid slots keep offset 0 (a valid tap) and
        // are never committed
        const int nslots = S * S;
        const int spg = (nslots + NG - 1) / NG;
        const int kdyn = (spg + kWave - 1) / kWave;
        // cell[k] = u | v << 16 of the slot's current cell (kNoCell: none yet;
        // u = 0xffff never is a footprint cell since footprints end below
        // the grid side, which is at most 65535)
        uint32_t cell[KMAX], offa[KMAX], offb[KMAX];
        bool sval[KMAX];
        float acc[KMAX][8];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int sl = k * kWave + lane;
            const int s = grp * spg + sl;
            sval[k] = (k < kdyn) && (sl < spg) && (s < nslots);
            cell[k] = kNoCell;
            offa[k] = 0u;
            offb[k] = 0u;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[k][q] = 0.0f;
        }

        auto commit = [&](float (&sums)[8], uint32_t cell_u, uint32_t cell_v) {
#pragma unroll
            for (int pol = 0; pol < 4; ++pol) {
                if (pol < npol) {
                    if constexpr (LDS) {
                        float2 *dst =
                            &region[(pol * RH + (int)(cell_v - cv0)) * RW + (int)(cell_u - cu0)];
                        atomicAdd(&dst->x, sums[2 * pol]);
                        atomicAdd(&dst->y, sums[2 * pol + 1]);
                    } else {
                        float *dst = grid + 2 * (((int64_t)pol * prm.nv + cell_v) * prm.nu + cell_u);
                        unsafeAtomicAdd(dst, sums[2 * pol]);
                        unsafeAtomicAdd(dst + 1, sums[2 * pol + 1]);
                    }
                }
            }
        };

        // one record: window update (only when its first cell changed) + FMAs
        uint32_t prev_kuv = 0xffffffffu;
        auto process = [&](const RecMeta m, const float4 v01, const float4 v23) {
            const uint32_t kuv = m.kuv;
            if (kuv != prev_kuv) {
                prev_kuv = kuv;
                const uint32_t ku = meta_ku(m), kv = meta_kv(m);
                bool moved[KMAX];
                bool any = false;
#pragma unroll
                for (int k = 0; k < KMAX; ++k) {
                    moved[k] = false;
                    if (k < kdyn) {
                        const uint32_t du = (cell[k] & 0xffffu) - ku, dv = (cell[k] >> 16) - kv;
                        moved[k] = sval[k] && (max(du, dv) >= (uint32_t)S);
                        any |= moved[k];
                    }
                }
                if (__ballot(any) != 0) {
                    const uint32_t kmu = ku % (uint32_t)S, kmv = kv % (uint32_t)S;
#pragma unroll
                    for (int k = 0; k < KMAX; ++k) {
                        if (k < kdyn && moved[k]) {
                            if (cell[k] != kNoCell) commit(acc[k], cell[k] & 0xffffu, cell[k] >> 16);
#pragma unroll
                            for (int q = 0; q < 8; ++q) acc[k][q] = 0.0f;
                            // slot (su, sv) owns the cells congruent to it mod S
                            const uint32_t sidx = (uint32_t)(grp * spg + k * kWave + lane);
                            const uint32_t sv = sidx / (uint32_t)S, su = sidx - sv * (uint32_t)S;
                            int du = (int)su - (int)kmu;
                            int dv = (int)sv - (int)kmv;
                            du += (du < 0) ? S : 0;
                            dv += (dv < 0) ? S : 0;
                            cell[k] = (ku + (uint32_t)du) | ((kv + (uint32_t)dv) << 16);
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < KMAX; ++k) {
                    if (k < kdyn) {
                        const uint32_t du = sval[k] ? (cell[k] & 0xffffu) - ku : 0u;
                        const uint32_t dv = sval[k] ? (cell[k] >> 16) - kv : 0u;
                        if constexpr (SEP) {
                            offa[k] = du * (uint32_t)beta * kElem;
                            offb[k] = dv * (uint32_t)beta * kElem;
                        } else {
                            offa[k] = (dv * (uint32_t)beta * rowlen + du * (uint32_t)beta) * kElem;
                        }
                    }
                }
            }
            const uint32_t ou1 = meta_ou(m) + 1, ov1 = meta_ov(m) + 1;
            // (kr + j ki)(vr + j vi) = kr vr - ki vi + j (kr vi + ki vr); the
            // conjugate table (w < 0) flips the sign of ki.
            const uint32_t flip = meta_conj(m) ? 0u : 0x80000000u;
            const float vr[4] = {v01.x, v01.z, v23.x, v23.z};
            const float vi[4] = {v01.y, v01.w, v23.y, v23.w};
            float va[4], vb[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                va[q] = __uint_as_float(__float_as_uint(vi[q]) ^ flip);
                vb[q] = __uint_as_float(__float_as_uint(vr[q]) ^ flip ^ 0x80000000u);
            }
            if constexpr (SEP) {
                const char *tu = tplane + (size_t)ou1 * kElem;
                const char *tv = tplane + (size_t)ov1 * kElem;
#pragma unroll
                for (int k = 0; k < KMAX; ++k) {
                    if (k < kdyn) {
                        const float w = TapTraits<TapT>::real((const TapT *)(tu + offa[k]), 0) *
                                        TapTraits<TapT>::real((const TapT *)(tv + offb[k]), 0);
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            acc[k][2 * q] = fmaf(w, vr[q], acc[k][2 * q]);
                            acc[k][2 * q + 1] = fmaf(w, vi[q], acc[k][2 * q + 1]);
                        }
                    }
                }
            } else {
                const char *tb = tplane + (size_t)(ov1 * rowlen + ou1) * kElem;
#pragma unroll
                for (int k = 0; k < KMAX; ++k) {
                    if (k < kdyn) {
                        const float2 w = TapTraits<TapT>::cplx((const TapT *)(tb + offa[k]), 0);
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            acc[k][2 * q] = fmaf(w.x, vr[q], fmaf(w.y, va[q], acc[k][2 * q]));
                            acc[k][2 * q + 1] = fmaf(w.x, vi[q], fmaf(w.y, vb[q], acc[k][2 * q + 1]));
                        }
                    }
                }
            }
        };

        const uint32_t len = ch.len;
        const uint32_t rb = ch.start + (uint32_t)(((uint64_t)len * split) / NSPLIT);
        const uint32_t re = ch.start + (uint32_t)(((uint64_t)len * (split + 1)) / NSPLIT);
        for (uint32_t r = rb; r < re; r += kBatch) {
            RecMeta mm[kBatch];
            float4 va4[kBatch], vb4[kBatch];
#pragma unroll
            for (int i = 0; i < kBatch; ++i) {
                const uint32_t ri = min(r + (uint32_t)i, re - 1);
                mm[i] = smeta[ri];
                va4[i] = svis[2 * (size_t)ri];
                vb4[i] = svis[2 * (size_t)ri + 1];
            }
            bool same = (r + kBatch <= re);
#pragma unroll
            for (int i = 0; i < kBatch; ++i) same = same && (mm[i].kuv == prev_kuv);
            if (!SEP && KMAX < 16 && same) {
                // the window does not move for the whole batch: issue all the
                // batch's tap loads before the first multiply-add
                float2 w[kBatch][KMAX];
#pragma unroll
                for (int i = 0; i < kBatch; ++i) {
                    const uint32_t ou1 = meta_ou(mm[i]) + 1, ov1 = meta_ov(mm[i]) + 1;
                    const char *tb = tplane + (size_t)(ov1 * rowlen + ou1) * kElem;
#pragma unroll
                    for (int k = 0; k < KMAX; ++k)
                        if (k < kdyn) w[i][k] = TapTraits<TapT>::cplx((const TapT *)(tb + offa[k]), 0);
                }
#pragma unroll
                for (int i = 0; i < kBatch; ++i) {
                    const uint32_t flip = meta_conj(mm[i]) ? 0u : 0x80000000u;
                    const float vr[4] = {va4[i].x, va4[i].z, vb4[i].x, vb4[i].z};
                    const float vi[4] = {va4[i].y, va4[i].w, vb4[i].y, vb4[i].w};
                    float xa[4], xb[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        xa[q] = __uint_as_float(__float_as_uint(vi[q]) ^ flip);
                        xb[q] = __uint_as_float(__float_as_uint(vr[q]) ^ flip ^ 0x80000000u);
                    }
#pragma unroll
                    for (int k = 0; k < KMAX; ++k) {
                        if (k < kdyn) {
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                acc[k][2 * q] = fmaf(w[i][k].x, vr[q], fmaf(w[i][k].y, xa[q], acc[k][2 * q]));
                                acc[k][2 * q + 1] =
                                    fmaf(w[i][k].x, vi[q], fmaf(w[i][k].y, xb[q], acc[k][2 * q + 1]));
                            }
                        }
                    }
                }
            } else {
#pragma unroll
                for (int i = 0; i < kBatch; ++i)
                    if (r + (uint32_t)i < re) process(mm[i], va4[i], vb4[i]);
            }
        }
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (k < kdyn && sval[k] && cell[k] != kNoCell) commit(acc[k], cell[k] & 0xffffu, cell[k] >> 16);

        if constexpr (LDS) {
            __syncthreads();
            const int n = npol * RH * RW;
            for (int i = threadIdx.x; i < n; i += kGroupThreads) {
                const float2 v = region[i];
                if (v.x != 0.0f || v.y != 0.0f) {
                    const int ru = i % RW;
                    const int t = i / RW;
                    const int rv = t % RH;
                    const int pol = t / RH;
                    float *dst = grid + 2 * (((int64_t)pol * prm.nv + cv0 + rv) * prm.nu + cu0 + ru);
                    unsafeAtomicAdd(dst, v.x);
                    unsafeAtomicAdd(dst + 1, v.y);
                }
            }
            __syncthreads();
        }
    }
}

// Gathers visibilities into sorted order, padded to 4 polarisations.
__global__ __launch_bounds__(256) void gather_vis_kernel(const int64_t *__restrict__ counters,
                                                         int64_t nrec,
                                                         const uint32_t *__restrict__ sperm,
                                                         const float2 *__restrict__ vis,
                                                         int32_t npol, float4 *__restrict__ svis) {
    const int64_t nvalid = counters[1];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvalid && i < nrec;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float2 *v = vis + (size_t)sperm[i] * npol;
        float2 x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = (q < npol) ? v[q] : make_float2(0.0f, 0.0f);
        svis[2 * i] = make_float4(x[0].x, x[0].y, x[1].x, x[1].y);
        svis[2 * i + 1] = make_float4(x[2].x, x[2].y, x[3].x, x[3].y);
    }
}

struct GridPtrs {
    const RecMeta *smeta;
    const float4 *svis;
    float *grid;
    const void *taps;
    const Chunk *chunks;
    const uint32_t *plane_cfirst;
    const PlaneLayout *planes;
};

template <int KMAX, int NG, bool SEP, typename TapT, bool LDS>
void launch_one(const GridPtrs &a, const GridParams &prm, size_t lds, hipStream_t stream,
                int blocks) {
    hipLaunchKernelGGL((grid_window_kernel<KMAX, NG, SEP, TapT, LDS>), dim3(blocks),
                       dim3(kGroupThreads), lds, stream, a.smeta, a.svis, a.grid,
                       (const TapT *)a.taps, a.chunks, a.plane_cfirst, a.planes, prm);
}

template <bool SEP, typename TapT>
hipError_t launch_class(int cls, const GridPtrs &a, const GridParams &prm, int smax, int tile,
                        hipStream_t stream, int blocks) {
    const size_t lds = (cls <= 2) ? sizeof(float2) * prm.npol * (size_t)(tile + smax - 1) *
                                        (size_t)(tile + smax - 1)
                                  : 0;
    switch (cls) {
    case 0: launch_one<1, 1, SEP, TapT, true>(a, prm, lds, stream, blocks); break;
    case 1: launch_one<4, 1, SEP, TapT, true>(a, prm, lds, stream, blocks); break;
    case 2: launch_one<8, 2, SEP, TapT, true>(a, prm, lds, stream, blocks); break;
    default: launch_one<16, 4, SEP, TapT, false>(a, prm, 0, stream, blocks); break;
    }
    return hipGetLastError();
}

template <bool SEP>
hipError_t launch_class_t(mg_dtype dt, int cls, const GridPtrs &a, const GridParams &prm,
                          int smax, int tile, hipStream_t stream, int blocks) {
    switch (dt) {
    case MG_F16: return launch_class<SEP, __half>(cls, a, prm, smax, tile, stream, blocks);
    case MG_BF16: return launch_class<SEP, __hip_bfloat16>(cls, a, prm, smax, tile, stream, blocks);
    default: return launch_class<SEP, float>(cls, a, prm, smax, tile, stream, blocks);
    }
}

}  // namespace

mg_status launch_grid(const PlanState &P, const void *vis, void *grid, hipStream_t stream) {
    if (P.nrec == 0) return MG_OK;
    float4 *svis = nullptr;
    hipError_t e = hipMallocAsync((void **)&svis, 2 * sizeof(float4) * (size_t)P.nrec, stream);
    if (e != hipSuccess) return set_error(MG_ENOMEM, "grid: gather buffer allocation failed");
    {
        int64_t nb = (P.nrec + 255) / 256;
        if (nb > 16384) nb = 16384;
        hipLaunchKernelGGL(gather_vis_kernel, dim3((unsigned)nb), dim3(256), 0, stream,
                           P.counters, P.nrec, P.sperm, (const float2 *)vis, P.geom.npol, svis);
    }
    GridPtrs a{P.smeta, svis, (float *)grid, P.taps, P.chunks, P.plane_cfirst, P.d_planes};
    GridParams prm{P.geom.npol, P.geom.nu, P.geom.nv, P.geom.beta, 0, 0};
    const bool sep = P.kind == MG_KERNEL_SEPARABLE;
    // one launch per run of consecutive planes of the same class
    const int np = P.nplanes_eff;
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
        const int blocks = 2048;
        e = sep ? launch_class_t<true>(P.tap_dtype, cls, a, prm, smax, P.planes[p0].T, stream,
                                       blocks)
                : launch_class_t<false>(P.tap_dtype, cls, a, prm, smax, P.planes[p0].T, stream,
                                        blocks);
        p0 = p1;
    }
    hipFreeAsync(svis, stream);
    if (e != hipSuccess) return set_error(MG_EDEVICE, std::string("grid kernels: ") + hipGetErrorString(e));
    return MG_OK;
}

}  // namespace mg
