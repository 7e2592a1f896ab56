// Degridding (gather) kernels: vis_out[r] = sum_{i,j} conj(w_ij) G[k_lo + (i, j)],
// the adjoint of the gridding map.
//
// Work unit: one chunk of cell-sorted records of one (plane, tile) bucket.
// The workgroup first copies the chunk's grid region (tile plus S-1 halo, all
// polarisations, interleaved per cell) from HBM into LDS with coalesced
// loads; then every lane takes whole records and sums their S x S footprint
// from LDS, so no cross-lane reduction and no atomics are needed.  For
// supports above 32 the region does not fit in LDS and lanes read the grid
// through the caches instead.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mg {

namespace {

struct DegridArgs {
    const RecMeta *smeta;
    const uint32_t *sperm;
    const float *grid;        // [npol][nv][nu] complex64
    float2 *vis_out;          // [nrec][npol]
    const void *taps;
    const Chunk *chunks;
    const uint32_t *plane_cfirst;
    const PlaneLayout *planes;
    int32_t npol, nu, nv, beta;
    int32_t p_lo, p_hi;
};

template <bool SEP, typename TapT, bool LDS>
__global__ __launch_bounds__(kGroupThreads) void degrid_kernel(DegridArgs a, DevGeom g) {
    extern __shared__ float2 region[];   // [row][col][pol]
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
        if constexpr (LDS) {
            const int n = npol * RH * RW;
            for (int i = threadIdx.x; i < n; i += kGroupThreads) {
                const int ru = i % RW;
                const int t = i / RW;
                const int rv = t % RH;
                const int pol = t / RH;
                const float2 v = *reinterpret_cast<const float2 *>(
                    a.grid + 2 * (((int64_t)pol * a.nv + cv0 + rv) * a.nu + cu0 + ru));
                region[(rv * RW + ru) * npol + pol] = v;
            }
            __syncthreads();
        }
        for (uint32_t i = threadIdx.x; i < ch.len; i += kGroupThreads) {
            const uint32_t r = ch.start + i;
            const RecMeta m = a.smeta[r];
            const uint32_t ku = meta_ku(m), kv = meta_kv(m);
            float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int j = 0; j < S; ++j) {
                float wv = 0.0f;
                if constexpr (SEP) wv = TapTraits<TapT>::real(taps, (int64_t)((m.toff >> 16) + j * a.beta));
                const int64_t trow = (int64_t)m.toff + (int64_t)j * a.beta * rowlen;
                for (int i2 = 0; i2 < S; ++i2) {
                    float wr, wi;
                    if constexpr (SEP) {
                        wr = TapTraits<TapT>::real(taps, (int64_t)((m.toff & 0xffffu) + i2 * a.beta)) * wv;
                        wi = 0.0f;
                    } else {
                        // records with w < 0 point into the conjugated bank
                        const float2 k = TapTraits<TapT>::cplx(taps, trow + i2 * a.beta);
                        wr = k.x;
                        wi = k.y;
                    }
#pragma unroll
                    for (int pol = 0; pol < 4; ++pol) {
                        if (pol < npol) {
                            float2 gv;
                            if constexpr (LDS) {
                                gv = region[((kv - cv0 + j) * RW + (ku - cu0 + i2)) * npol + pol];
                            } else {
                                gv = *reinterpret_cast<const float2 *>(
                                    a.grid + 2 * (((int64_t)pol * a.nv + kv + j) * a.nu + ku + i2));
                            }
                            // conj(w) * G = (wr gr + wi gi) + j (wr gi - wi gr)
                            acc[2 * pol] = fmaf(wr, gv.x, fmaf(wi, gv.y, acc[2 * pol]));
                            acc[2 * pol + 1] = fmaf(wr, gv.y, fmaf(-wi, gv.x, acc[2 * pol + 1]));
                        }
                    }
                }
            }
            float2 *out = a.vis_out + (size_t)a.sperm[r] * npol;
#pragma unroll
            for (int pol = 0; pol < 4; ++pol)
                if (pol < npol) out[pol] = make_float2(acc[2 * pol], acc[2 * pol + 1]);
        }
        if constexpr (LDS) __syncthreads();
    }
}

// Zero the outputs of skipped records (and everything, before valid records
// overwrite theirs).
__global__ __launch_bounds__(256) void zero_vis_kernel(float2 *__restrict__ v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v[i] = make_float2(0.0f, 0.0f);
}

template <bool SEP, typename TapT>
hipError_t launch_deg(int cls, const DegridArgs &a, const DevGeom &g, int smax, int tile,
                      hipStream_t stream, int blocks) {
    if (cls <= 2) {
        const size_t lds = sizeof(float2) * a.npol * (size_t)(tile + smax - 1) *
                           (size_t)(tile + smax - 1);
        hipLaunchKernelGGL((degrid_kernel<SEP, TapT, true>), dim3(blocks), dim3(kGroupThreads),
                           lds, stream, a, g);
    } else {
        hipLaunchKernelGGL((degrid_kernel<SEP, TapT, false>), dim3(blocks), dim3(kGroupThreads),
                           0, stream, a, g);
    }
    return hipGetLastError();
}

template <bool SEP>
hipError_t launch_deg_t(mg_dtype dt, int cls, const DegridArgs &a, const DevGeom &g, int smax,
                        int tile, hipStream_t stream, int blocks) {
    switch (dt) {
    case MG_F16:
        return launch_deg<SEP, __half>(cls, a, g, smax, tile, stream, blocks);
    case MG_BF16:
        return launch_deg<SEP, __hip_bfloat16>(cls, a, g, smax, tile, stream, blocks);
    default:
        return launch_deg<SEP, float>(cls, a, g, smax, tile, stream, blocks);
    }
}

}  // namespace

mg_status launch_degrid(const PlanState &P, const void *grid, void *vis_out, hipStream_t stream) {
    const int64_t nv = P.nrec * P.geom.npol;
    if (nv == 0) return MG_OK;
    {
        int64_t nb = (nv + 255) / 256;
        if (nb > 16384) nb = 16384;
        hipLaunchKernelGGL(zero_vis_kernel, dim3((unsigned)nb), dim3(256), 0, stream,
                           (float2 *)vis_out, nv);
    }
    DegridArgs a;
    a.smeta = P.smeta;
    a.sperm = P.sperm;
    a.grid = (const float *)grid;
    a.vis_out = (float2 *)vis_out;
    a.taps = P.taps;
    a.chunks = P.chunks;
    a.plane_cfirst = P.plane_cfirst;
    a.planes = P.d_planes;
    a.npol = P.geom.npol;
    a.nu = P.geom.nu;
    a.nv = P.geom.nv;
    a.beta = P.geom.beta;
    const bool sep = P.kind == MG_KERNEL_SEPARABLE;
    hipError_t e = hipGetLastError();
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
        e = sep ? launch_deg_t<true>(P.tap_dtype, cls, a, P.geom, smax, P.planes[p0].T, stream, 2048)
                : launch_deg_t<false>(P.tap_dtype, cls, a, P.geom, smax, P.planes[p0].T, stream,
                                      2048);
        p0 = p1;
    }
    if (e != hipSuccess) return set_error(MG_EDEVICE, std::string("degrid kernels: ") + hipGetErrorString(e));
    return MG_OK;
}

}  // namespace mg
