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

struct GridArgs {
    const RecMeta *smeta;     // sorted records
    const float4 *svis;       // [nvalid][2] : 4 polarisations, gathered in sorted order
    float *grid;              // [npol][nv][nu] complex64
    const void *taps;
    const Chunk *chunks;
    const uint32_t *plane_cfirst;
    const PlaneLayout *planes;
    int32_t npol, nu, nv, beta;
    int32_t p_lo, p_hi;       // planes handled by this launch
};

template <typename TapT, bool SEP>
__device__ inline float2 load_weight(const TapT *taps, int64_t poff, int rowlen, int beta,
                                     uint32_t ou1, uint32_t ov1, uint32_t du, uint32_t dv) {
    if constexpr (SEP) {
        float wu = TapTraits<TapT>::real(taps, (int64_t)(ou1 + du * beta));
        float wv = TapTraits<TapT>::real(taps, (int64_t)(ov1 + dv * beta));
        return make_float2(wu * wv, 0.0f);
    } else {
        int64_t t = poff + (int64_t)(ov1 + dv * beta) * rowlen + (ou1 + du * beta);
        return TapTraits<TapT>::cplx(taps, t);
    }
}

// KMAX: slots per lane (compile-time upper bound); NG: slot groups (waves
// that share one chunk's records but own different slots); LDS: commit into
// the shared LDS region (else straight into the grid).
template <int KMAX, int NG, bool SEP, typename TapT, bool LDS>
__global__ __launch_bounds__(kGroupThreads) void grid_window_kernel(GridArgs a, DevGeom g) {
    extern __shared__ float2 region[];
    constexpr int NSPLIT = kWavesPerGroup / NG;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int grp = wave % NG;
    const int split = wave / NG;
    const TapT *taps = (const TapT *)a.taps;
    const int npol = a.npol;
    const uint32_t c_begin = a.plane_cfirst[a.p_lo];
    const uint32_t c_end = a.plane_cfirst[a.p_hi];

    for (uint32_t c = c_begin + blockIdx.x; c < c_end; c += gridDim.x) {
        const Chunk ch = a.chunks[c];
        int p = a.p_lo;
        while (p + 1 < a.p_hi && (int64_t)ch.bucket >= a.planes[p + 1].base) ++p;
        const PlaneLayout pl = a.planes[p];
        const int S = pl.S;
        const uint32_t local = ch.bucket - (uint32_t)pl.base;
        const uint32_t tu0 = (local % (uint32_t)pl.ntu) << pl.log2T;
        const uint32_t tv0 = (local / (uint32_t)pl.ntu) << pl.log2T;
        const uint32_t cu0 = tu0 + (ch.bbox & 0xffu);
        const uint32_t cv0 = tv0 + ((ch.bbox >> 16) & 0xffu);
        const int RW = (int)((ch.bbox >> 8) & 0xffu) - (int)(ch.bbox & 0xffu) + S;
        const int RH = (int)(ch.bbox >> 24) - (int)((ch.bbox >> 16) & 0xffu) + S;
        const int rowlen = a.beta * S + 1;
        const int64_t poff = SEP ? 0 : g.plane_offset[p];

        if constexpr (LDS) {
            for (int i = threadIdx.x; i < npol * RH * RW; i += kGroupThreads)
                region[i] = make_float2(0.0f, 0.0f);
            __syncthreads();
        }

        // slots of this wave
        const int nslots = S * S;
        const int spg = (nslots + NG - 1) / NG;           // slots per group
        const int kdyn = (spg + kWave - 1) / kWave;        // <= KMAX by class choice
        uint32_t cu[KMAX], cv[KMAX], su[KMAX], sv[KMAX];
        bool sval[KMAX];
        float acc[KMAX][8];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            int sl = k * kWave + lane;
            int s = grp * spg + sl;
            sval[k] = (k < kdyn) && (sl < spg) && (s < nslots);
            su[k] = sval[k] ? (uint32_t)(s % S) : 0u;
            sv[k] = sval[k] ? (uint32_t)(s / S) : 0u;
            cu[k] = kNoCell;
            cv[k] = kNoCell;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[k][q] = 0.0f;
        }

        // Adds one slot's sums to its cell (LDS region or grid).
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
                        float *dst = a.grid + 2 * (((int64_t)pol * a.nv + cell_v) * a.nu + cell_u);
                        unsafeAtomicAdd(dst, sums[2 * pol]);
                        unsafeAtomicAdd(dst + 1, sums[2 * pol + 1]);
                    }
                }
            }
        };

        const uint32_t len = ch.len;
        const uint32_t rb = ch.start + (uint32_t)(((uint64_t)len * split) / NSPLIT);
        const uint32_t re = ch.start + (uint32_t)(((uint64_t)len * (split + 1)) / NSPLIT);
        for (uint32_t r = rb; r < re; ++r) {
            const RecMeta m = a.smeta[r];
            const float4 v01 = a.svis[2 * (size_t)r];
            const float4 v23 = a.svis[2 * (size_t)r + 1];
            const uint32_t ku = meta_ku(m), kv = meta_kv(m);
            const uint32_t ou1 = meta_ou(m) + 1, ov1 = meta_ov(m) + 1;
            const bool cj = meta_conj(m) != 0;
            float vr[4] = {v01.x, v01.z, v23.x, v23.z};
            float vi[4] = {v01.y, v01.w, v23.y, v23.w};
            // (kr + j ki)(vr + j vi) = kr vr - ki vi + j (kr vi + ki vr);
            // the conjugate table for w < 0 flips the sign of ki.
            float va[4], vb[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                va[q] = cj ? vi[q] : -vi[q];
                vb[q] = cj ? -vr[q] : vr[q];
            }

            bool moved[KMAX];
            bool any = false;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                if (k < kdyn) {
                    uint32_t du = cu[k] - ku, dv = cv[k] - kv;
                    moved[k] = sval[k] && (du >= (uint32_t)S || dv >= (uint32_t)S);
                    any |= moved[k];
                } else {
                    moved[k] = false;
                }
            }
            if (__ballot(any) != 0) {
                const uint32_t kmu = ku % (uint32_t)S, kmv = kv % (uint32_t)S;
#pragma unroll
                for (int k = 0; k < KMAX; ++k) {
                    if (k < kdyn && moved[k]) {
                        if (cu[k] != kNoCell) commit(acc[k], cu[k], cv[k]);
#pragma unroll
                        for (int q = 0; q < 8; ++q) acc[k][q] = 0.0f;
                        int du = (int)su[k] - (int)kmu;
                        int dv = (int)sv[k] - (int)kmv;
                        du += (du < 0) ? S : 0;
                        dv += (dv < 0) ? S : 0;
                        cu[k] = ku + (uint32_t)du;
                        cv[k] = kv + (uint32_t)dv;
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                if (k < kdyn && sval[k]) {
                    const uint32_t du = cu[k] - ku, dv = cv[k] - kv;
                    const float2 w = load_weight<TapT, SEP>(taps, poff, rowlen, a.beta, ou1, ov1,
                                                            du, dv);
                    if constexpr (SEP) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            acc[k][2 * q] = fmaf(w.x, vr[q], acc[k][2 * q]);
                            acc[k][2 * q + 1] = fmaf(w.x, vi[q], acc[k][2 * q + 1]);
                        }
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            acc[k][2 * q] = fmaf(w.x, vr[q], fmaf(w.y, va[q], acc[k][2 * q]));
                            acc[k][2 * q + 1] =
                                fmaf(w.x, vi[q], fmaf(w.y, vb[q], acc[k][2 * q + 1]));
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            if (k < kdyn && sval[k] && cu[k] != kNoCell) commit(acc[k], cu[k], cv[k]);

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
                    float *dst = a.grid + 2 * (((int64_t)pol * a.nv + cv0 + rv) * a.nu + cu0 + ru);
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

template <bool SEP, typename TapT>
hipError_t launch_class(int cls, const GridArgs &a, const DevGeom &g, int smax, int tile,
                        hipStream_t stream, int blocks) {
    const size_t lds = (cls <= 2) ? sizeof(float2) * a.npol * (size_t)(tile + smax - 1) *
                                        (size_t)(tile + smax - 1)
                                  : 0;
    switch (cls) {
    case 0:
        hipLaunchKernelGGL((grid_window_kernel<1, 1, SEP, TapT, true>), dim3(blocks),
                           dim3(kGroupThreads), lds, stream, a, g);
        break;
    case 1:
        hipLaunchKernelGGL((grid_window_kernel<4, 1, SEP, TapT, true>), dim3(blocks),
                           dim3(kGroupThreads), lds, stream, a, g);
        break;
    case 2:
        hipLaunchKernelGGL((grid_window_kernel<16, 1, SEP, TapT, true>), dim3(blocks),
                           dim3(kGroupThreads), lds, stream, a, g);
        break;
    default:
        hipLaunchKernelGGL((grid_window_kernel<16, 4, SEP, TapT, false>), dim3(blocks),
                           dim3(kGroupThreads), 0, stream, a, g);
        break;
    }
    return hipGetLastError();
}

template <bool SEP>
hipError_t launch_class_t(mg_dtype dt, int cls, const GridArgs &a, const DevGeom &g, int smax,
                          int tile, hipStream_t stream, int blocks) {
    switch (dt) {
    case MG_F16:
        return launch_class<SEP, __half>(cls, a, g, smax, tile, stream, blocks);
    case MG_BF16:
        return launch_class<SEP, __hip_bfloat16>(cls, a, g, smax, tile, stream, blocks);
    default:
        return launch_class<SEP, float>(cls, a, g, smax, tile, stream, blocks);
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
    GridArgs a;
    a.smeta = P.smeta;
    a.svis = svis;
    a.grid = (float *)grid;
    a.taps = P.taps;
    a.chunks = P.chunks;
    a.plane_cfirst = P.plane_cfirst;
    a.planes = P.d_planes;
    a.npol = P.geom.npol;
    a.nu = P.geom.nu;
    a.nv = P.geom.nv;
    a.beta = P.geom.beta;
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
        a.p_lo = p0;
        a.p_hi = p1;
        const int cls = P.planes[p0].cls;
        const int blocks = 2048;
        e = sep ? launch_class_t<true>(P.tap_dtype, cls, a, P.geom, smax, P.planes[p0].T, stream,
                                       blocks)
                : launch_class_t<false>(P.tap_dtype, cls, a, P.geom, smax, P.planes[p0].T, stream,
                                        blocks);
        p0 = p1;
    }
    hipFreeAsync(svis, stream);
    if (e != hipSuccess) return set_error(MG_EDEVICE, std::string("grid kernels: ") + hipGetErrorString(e));
    return MG_OK;
}

}  // namespace mg
