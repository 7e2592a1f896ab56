// Shared definitions of the migrid HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "../../include/migrid.h"

namespace mg {

constexpr int kWave = 64;
constexpr int kMaxPlanes = 128;
constexpr int kMaxSupport = 64;
constexpr int kMaxBeta = 256;
constexpr int kMaxN = 65535;

// Geometry and kernel description as the device sees it (passed by value).
struct DevGeom {
    int32_t nu, nv, npol, beta;
    double scale_u, scale_v;
    int32_t nplanes;         // 0 = separable
    int32_t support;         // separable S
    double inv_dw;
    int32_t plane_support[kMaxPlanes];
    int64_t plane_offset[kMaxPlanes];   // element offset of plane p (in the
                                        // plan's table once a plan owns it)
    int64_t conj_base;                  // W-projection: element offset of the
                                        // conjugated copy of the bank
    int32_t layers;                     // W-stacking: layer count (0 = none);
    int32_t layer_nv;                   // rows of one layer (nv = layers x layer_nv)
};

// A plan keeps its own copy of the tap table in phase-major order: for each
// oversampling phase o (0 <= o < beta) the S taps o + 1 + j beta
// (j = 0 .. S-1) of an axis are stored one after another, so the taps a
// record needs are contiguous.  W-projection plane p: beta^2 blocks of
// S x S complex taps, block (o_v, o_u) holding
// bank[(o_v + 1 + j beta) * (beta S + 1) + (o_u + 1 + i beta)] at j S + i;
// separable: beta blocks of S taps.
//
// Per-record packed index, 8 bytes:
//   kuv  = k_lo_u | k_lo_v << 16
//   toff = W-projection: element of the plan's table holding the record's
//            first tap, plane offset + (o_v beta + o_u) S^2, inside the
//            conjugated copy of the table for w < 0;
//          separable: o_u S | (o_v S) << 16.
// The gridders then address tap (i, j) as toff + j S + i (or toff_u + i,
// toff_v + j) without decoding anything else.
struct RecMeta {
    uint32_t kuv;
    uint32_t toff;
};

__host__ __device__ inline uint32_t meta_ku(RecMeta m) { return m.kuv & 0xffffu; }
__host__ __device__ inline uint32_t meta_kv(RecMeta m) { return m.kuv >> 16; }

// One result of the index rule.
struct RecIndex {
    int32_t ku, kv, ou, ov, plane, S, conj, valid;
};

// One axis of the index rule, in FP64 with every operation rounded as
// written (no contraction into fused multiply-add), so that the GPU and any
// other implementation of the same rule agree bit for bit.
__device__ inline bool index_axis(double coord, double scale, int32_t n, int32_t beta, int32_t S,
                                  int32_t *k_lo, int32_t *o) {
#pragma clang fp contract(off)
    double x = coord * scale;
    x = x + (double)(n / 2);
    double xb = x * (double)beta;
    xb = xb + 0.5;
    double fq = floor(xb);
    if (!(fabs(fq) < 4.0e15)) return false;
    int64_t q = (int64_t)fq;
    int64_t half = (int64_t)beta * S / 2;
    // k = floor((q - half) / beta) + 1 lies in [0, n - S] exactly when
    // -beta <= q - half < beta * (n - S); inside that range the shifted
    // numerator is non-negative and below 2^31, so one unsigned 32-bit
    // division gives k (no 64-bit division).
    const int64_t d = q - half;
    const bool ok = (d >= -(int64_t)beta) && (d < (int64_t)beta * ((int64_t)n - S));
    const uint32_t k = ok ? (uint32_t)(d + beta) / (uint32_t)beta : 0u;
    const int64_t t0 = (int64_t)k * beta - d;
    *k_lo = ok ? (int32_t)k : 0;
    *o = ok ? (int32_t)(t0 - 1) : 0;
    return ok;
}

template <typename T>
__device__ inline RecIndex index_record(const DevGeom &g, T u_, T v_, T w_) {
#pragma clang fp contract(off)
    RecIndex r;
    r.ku = r.kv = r.ou = r.ov = 0;
    r.plane = -1;
    r.conj = 0;
    r.valid = 0;
    double u = (double)u_, v = (double)v_, w = (double)w_;
    r.S = g.support;
    if (!(isfinite(u) && isfinite(v) && isfinite(w))) return r;
    if (g.nplanes > 0) {
        double a = fabs(w) * g.inv_dw;
        a = a + 0.5;
        double fp = floor(a);
        int32_t p = (fp >= (double)(g.nplanes - 1)) ? g.nplanes - 1 : (int32_t)fp;
        r.plane = p;
        r.conj = (w < 0.0) ? 1 : 0;
        r.S = g.plane_support[p];
    }
    bool okU = index_axis(u, g.scale_u, g.nu, g.beta, r.S, &r.ku, &r.ou);
    if (g.layers > 0) {
        // W-stacking: layer j = floor(w inv_dw + L/2) clamped to [0, L-1]
        // (centred on w_j = (j - (L-1)/2) dw); the record is placed on its
        // layer's own grid, which occupies rows j layer_nv .. (j+1) layer_nv - 1
        double a = w * g.inv_dw;
        a = a + 0.5 * (double)g.layers;
        const double fj = floor(a);
        const int32_t j = fj <= 0.0 ? 0
                          : (fj >= (double)(g.layers - 1) ? g.layers - 1 : (int32_t)fj);
        bool okV = index_axis(v, g.scale_v, g.layer_nv, g.beta, r.S, &r.kv, &r.ov);
        r.kv += j * g.layer_nv;
        r.valid = (okU && okV) ? 1 : 0;
        return r;
    }
    bool okV = index_axis(v, g.scale_v, g.nv, g.beta, r.S, &r.kv, &r.ov);
    r.valid = (okU && okV) ? 1 : 0;
    return r;
}

__device__ inline RecMeta pack_meta(const DevGeom &g, const RecIndex &r) {
    RecMeta m;
    m.kuv = (uint32_t)r.ku | ((uint32_t)r.kv << 16);
    if (g.nplanes == 0) {
        m.toff = (uint32_t)(r.ou * r.S) | ((uint32_t)(r.ov * r.S) << 16);
    } else {
        const int64_t p = r.plane < 0 ? 0 : r.plane;
        m.toff = (uint32_t)(g.plane_offset[p] + ((int64_t)r.ov * g.beta + r.ou) * r.S * r.S +
                            (r.conj ? g.conj_base : 0));
    }
    return m;
}

// Tap loads: a tap table element of type TapT expanded to FP32.
template <typename TapT> struct TapTraits;
template <> struct TapTraits<float> {
    static __device__ inline float real(const float *p, int64_t i) { return p[i]; }
    static __device__ inline float2 cplx(const float *p, int64_t i) {
        return *reinterpret_cast<const float2 *>(p + 2 * i);
    }
};
template <> struct TapTraits<__half> {
    static __device__ inline float real(const __half *p, int64_t i) { return __half2float(p[i]); }
    static __device__ inline float2 cplx(const __half *p, int64_t i) {
        __half2 h = *reinterpret_cast<const __half2 *>(p + 2 * i);
        return __half22float2(h);
    }
};
template <> struct TapTraits<__hip_bfloat16> {
    static __device__ inline float real(const __hip_bfloat16 *p, int64_t i) {
        return __bfloat162float(p[i]);
    }
    static __device__ inline float2 cplx(const __hip_bfloat16 *p, int64_t i) {
        uint32_t bits = *reinterpret_cast<const uint32_t *>(p + 2 * i);
        float2 f;
        f.x = __uint_as_float(bits << 16);
        f.y = __uint_as_float(bits & 0xffff0000u);
        return f;
    }
};

// Wave-aggregated counter increment.  Lanes with `active` add 1 to
// counters[key]; lanes sharing a key are served by one atomic issued by the
// lowest of them.  Returns, for each active lane, the counter's value before
// the group's add plus the lane's rank within its group (so the lanes of a
// group get consecutive values in lane order).  Records arrive in
// measurement-set order, where consecutive channels of a baseline share a
// bucket, so one atomic per group replaces up to 64 serialised ones.  The
// groups are formed first; then every group's leader issues its atomic in
// one vector instruction, so the wave waits for one atomic round trip.
__device__ inline uint32_t wave_counter_add(uint32_t *counters, uint32_t key, bool active,
                                            bool need_value) {
    const int lane = threadIdx.x & 63;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t pending = __ballot(active);
    int leader = lane;      // this lane's group leader
    uint32_t rank = 0;      // position within the group
    uint32_t count = 0;     // group size (leaders)
    while (pending) {
        const int l = __builtin_ctzll(pending);
        const uint32_t lkey = __builtin_amdgcn_readlane(key, l);
        const uint64_t group = __ballot(active && key == lkey) & pending;
        if ((group >> lane) & 1ull) {
            leader = l;
            rank = (uint32_t)__popcll(group & lt);
        }
        if (lane == l) count = (uint32_t)__popcll(group);
        pending &= ~group;
    }
    uint32_t base = 0;
    if (active && leader == lane) {
        if (need_value) base = atomicAdd(&counters[key], count);
        else atomicAdd(&counters[key], count);
    }
    if (!need_value) return 0;
    base = (uint32_t)__shfl((int)base, leader, 64);
    return base + rank;
}

// Uniform (scalar) broadcast helpers.
__device__ inline uint32_t uniform_u32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline float uniform_f32(float x) {
    return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(x)));
}

}  // namespace mg
