// W-projection kernel bank builder.
//
// Plane p of the bank tabulates, at 1/beta cells over its support S_p, the
// GCF convolved with the transform of the inverse W-term (Section 1.7.1,
// W-projection; Section 1.3 for the W-term g_w and gbar_w = 1 / g_w):
//     K_p = F[ c(l) c(m) gbar_{w_p}(l, m) ],
//     gbar_w(l, m) = exp(+j2pi w (sqrt(1 - l^2 - m^2) - 1)),
// with c the image-domain taper of the separable GCF C (c = F^-1 C) and F
// the transform with exp(-j2pi (ul + vm)).  Discretisation: an M x M image
// grid, M = 2 beta S_p, of spacing beta / M field units (so its transform
// has uv spacing 1/beta cells and spans 2 S_p cells), physical direction
// cosines = field units x fov; the central beta S_p + 1 samples per axis
// are kept.  Steps, all in FP64 on the device:
//   taper_kernel   c[i] = (1/M) sum_tau T[tau] cos(2pi tau i / M), i centred
//                  (T symmetric, so the inverse DFT is real)
//   screen_kernel  img = c[i] c[j] gbar(l_i, m_j), written straight in the
//                  transform's order (index 0 = centre)
//   the platform library's batched Z2Z forward FFT, one batch per distinct M
//   maxabs_kernel  largest |K| over every plane's kept samples
//   store_kernel   bank = K / max, converted to the output tap format, row
//                  (v offset) major.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "internal.h"

namespace mg {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

__global__ __launch_bounds__(256) void taper_kernel(int32_t M, int32_t base_len,
                                                    const double *__restrict__ T,
                                                    double *__restrict__ c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int ic = i - M / 2;
    const int h = (base_len - 1) / 2;
    double s = 0.0;
    for (int t = 0; t < base_len; ++t) {
        // tau i mod M keeps the cosine argument small and exact
        const int64_t ph = ((int64_t)(t - h) * ic) % M;
        s += T[t] * cos(kTwoPi * (double)ph / (double)M);
    }
    c[i] = s / (double)M;
}

// One plane: img[k1][k2], k in transform order (signed index k or k - M).
__global__ __launch_bounds__(256) void screen_kernel(int32_t M, int32_t beta, double w,
                                                     double fov, const double *__restrict__ c,
                                                     double2 *__restrict__ img) {
    const int64_t n = (int64_t)M * M;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int k1 = (int)(k / M), k2 = (int)(k - (int64_t)k1 * M);
        const int i = k1 < M / 2 ? k1 : k1 - M;   // signed (centred) index
        const int j = k2 < M / 2 ? k2 : k2 - M;
        const double l = (double)i * ((double)beta / (double)M) * fov;
        const double m = (double)j * ((double)beta / (double)M) * fov;
        const double r2 = l * l + m * m;
        const double nn = r2 < 1.0 ? sqrt(1.0 - r2) : 0.0;
        double sn, cs;
        sincos(kTwoPi * w * (nn - 1.0), &sn, &cs);
        const double a = c[i + M / 2] * c[j + M / 2];
        img[k] = make_double2(a * cs, a * sn);
    }
}

struct PlaneJob {
    int32_t M, S;
    int64_t img_off;     // complex elements into the FFT buffer
    int64_t bank_off;    // complex elements into the bank
};

// Kept sample (ta, tb) of plane p sits at transform index (t - beta S / 2) mod M.
__device__ inline int64_t kept_index(int ta, int tb, int M, int half) {
    const int a = ((ta - half) % M + M) % M;
    const int b = ((tb - half) % M + M) % M;
    return (int64_t)a * M + b;
}

__global__ __launch_bounds__(256) void clear_max_kernel(unsigned long long *mx) { *mx = 0ull; }

__global__ __launch_bounds__(256) void maxabs_kernel(const PlaneJob *__restrict__ jobs,
                                                     int32_t beta, const double2 *__restrict__ buf,
                                                     unsigned long long *mx) {
    const PlaneJob jb = jobs[blockIdx.y];
    const int E = beta * jb.S + 1;
    const int half = beta * jb.S / 2;
    double best = 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < E * E; t += gridDim.x * blockDim.x) {
        const int ta = t / E, tb = t - ta * E;
        const double2 v = buf[jb.img_off + kept_index(ta, tb, jb.M, half)];
        best = fmax(best, sqrt(v.x * v.x + v.y * v.y));
    }
    // magnitudes are non-negative, so their bit patterns order like the values
    for (int o = 32; o > 0; o >>= 1)
        best = fmax(best, __shfl_xor(best, o));
    if ((threadIdx.x & 63) == 0) atomicMax(mx, (unsigned long long)__double_as_longlong(best));
}

template <typename OutT> __device__ inline void store_tap(OutT *bank, int64_t i, double re, double im);
template <> __device__ inline void store_tap<float>(float *bank, int64_t i, double re, double im) {
    bank[2 * i] = (float)re;
    bank[2 * i + 1] = (float)im;
}
// FP16 and BF16: rounded to FP32, then to the nearest value of the format
// (ties to even)
template <> __device__ inline void store_tap<__half>(__half *bank, int64_t i, double re, double im) {
    bank[2 * i] = __float2half((float)re);
    bank[2 * i + 1] = __float2half((float)im);
}
template <>
__device__ inline void store_tap<__hip_bfloat16>(__hip_bfloat16 *bank, int64_t i, double re,
                                                 double im) {
    bank[2 * i] = __float2bfloat16((float)re);
    bank[2 * i + 1] = __float2bfloat16((float)im);
}

template <typename OutT>
__global__ __launch_bounds__(256) void store_kernel(const PlaneJob *__restrict__ jobs, int32_t beta,
                                                    const double2 *__restrict__ buf,
                                                    const unsigned long long *mx,
                                                    OutT *__restrict__ bank) {
    const PlaneJob jb = jobs[blockIdx.y];
    const int E = beta * jb.S + 1;
    const int half = beta * jb.S / 2;
    const double m = __longlong_as_double((long long)*mx);
    const double inv = m > 0.0 ? 1.0 / m : 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < E * E; t += gridDim.x * blockDim.x) {
        const int ta = t / E, tb = t - ta * E;
        const double2 v = buf[jb.img_off + kept_index(ta, tb, jb.M, half)];
        store_tap<OutT>(bank, jb.bank_off + t, v.x * inv, v.y * inv);
    }
}

struct Layout {
    std::vector<PlaneJob> jobs;
    std::map<int, std::vector<int>> by_m;   // M -> planes (FFT batch order)
    int64_t bank_elems = 0;
    int64_t img_elems = 0;
    int64_t taper_elems = 0;
    size_t bytes = 0;
    size_t off_img = 0, off_taper = 0, off_jobs = 0, off_max = 0;
};

mg_status make_layout(int32_t nplanes, const int32_t *sup, int32_t beta, Layout &L) {
    if (nplanes < 1 || nplanes > kMaxPlanes) return set_error(MG_EINVAL, "nplanes must be in 1..128");
    if (!sup) return set_error(MG_EINVAL, "null plane supports");
    if (beta < 1 || beta > kMaxBeta) return set_error(MG_EINVAL, "beta must be in 1..256");
    L.jobs.resize(nplanes);
    for (int p = 0; p < nplanes; ++p) {
        const int S = sup[p];
        if (S < 1 || S > kMaxSupport) return set_error(MG_EINVAL, "plane support must be in 1..64");
        if (((int64_t)beta * S) % 2) return set_error(MG_EINVAL, "beta * support must be even");
        // the FP64 image grid of a plane is (2 beta S)^2 x 16 bytes
        if ((int64_t)beta * S > 4096) return set_error(MG_EINVAL, "beta * support must be <= 4096");
        L.jobs[p].S = S;
        L.jobs[p].M = 2 * beta * S;
        L.jobs[p].bank_off = L.bank_elems;
        L.bank_elems += (int64_t)(beta * S + 1) * (beta * S + 1);
        L.by_m[L.jobs[p].M].push_back(p);
    }
    // FFT buffer: the planes of one M contiguous (one batched transform)
    for (auto &kv : L.by_m)
        for (int p : kv.second) {
            L.jobs[p].img_off = L.img_elems;
            L.img_elems += (int64_t)kv.first * kv.first;
            L.taper_elems += kv.first;
        }
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t at = off;
        off += arena_round(b);
        return at;
    };
    L.off_img = take(sizeof(double2) * (size_t)L.img_elems);
    L.off_taper = take(sizeof(double) * (size_t)L.taper_elems);
    L.off_jobs = take(sizeof(PlaneJob) * (size_t)nplanes);
    L.off_max = take(sizeof(unsigned long long));
    L.bytes = off;
    return MG_OK;
}

}  // namespace
}  // namespace mg

using namespace mg;

extern "C" {

mg_status mg_wkernel_bank_size(int32_t nplanes, const int32_t *plane_support, int32_t beta,
                               int64_t *bank_elems, size_t *workspace_bytes) {
    if (!bank_elems || !workspace_bytes) return set_error(MG_EINVAL, "null output");
    Layout L;
    const mg_status st = make_layout(nplanes, plane_support, beta, L);
    if (st != MG_OK) return st;
    *bank_elems = L.bank_elems;
    *workspace_bytes = L.bytes;
    return MG_OK;
}

mg_status mg_wkernel_bank(int32_t nplanes, const int32_t *plane_support, const double *plane_w,
                          int32_t beta, int32_t base_len, const double *base_taps, double fov,
                          mg_dtype out_dtype, void *bank, int64_t *plane_offset, void *workspace,
                          size_t workspace_bytes, hipStream_t stream) {
    Layout L;
    mg_status st = make_layout(nplanes, plane_support, beta, L);
    if (st != MG_OK) return st;
    if (!plane_w || !base_taps || !bank || !plane_offset || !workspace)
        return set_error(MG_EINVAL, "null argument");
    if (workspace_bytes < L.bytes) return set_error(MG_EINVAL, "workspace too small");
    if (base_len < 1 || (base_len % 2) == 0) return set_error(MG_EINVAL, "base table length must be odd");
    if (!(fov > 0.0) || !std::isfinite(fov)) return set_error(MG_EINVAL, "fov must be positive");
    if (out_dtype != MG_F32 && out_dtype != MG_F16 && out_dtype != MG_BF16)
        return set_error(MG_EINVAL, "bank dtype must be MG_F32, MG_F16 or MG_BF16");
    for (int p = 0; p < nplanes; ++p) {
        if (!std::isfinite(plane_w[p])) return set_error(MG_EINVAL, "plane w must be finite");
        if (base_len > beta * plane_support[p] + 1)
            return set_error(MG_EINVAL, "plane support narrower than the base kernel");
    }
    char *ws = static_cast<char *>(workspace);
    double2 *img = reinterpret_cast<double2 *>(ws + L.off_img);
    double *taper = reinterpret_cast<double *>(ws + L.off_taper);
    PlaneJob *djobs = reinterpret_cast<PlaneJob *>(ws + L.off_jobs);
    unsigned long long *mx = reinterpret_cast<unsigned long long *>(ws + L.off_max);

    hipError_t e = hipMemcpyAsync(djobs, L.jobs.data(), sizeof(PlaneJob) * nplanes,
                                  hipMemcpyHostToDevice, stream);
    // plan every distinct size first (plan creation synchronises the device)
    std::vector<std::pair<int, hipfftHandle>> plans;
    mg_status out = MG_OK;
    for (auto &kv : L.by_m) {
        hipfftHandle h = 0;
        int dims[2] = {kv.first, kv.first};
        const int dist = kv.first * kv.first;
        const hipfftResult r = hipfftPlanMany(&h, 2, dims, nullptr, 1, dist, nullptr, 1, dist,
                                              HIPFFT_Z2Z, (int)kv.second.size());
        if (r != HIPFFT_SUCCESS) {
            out = set_error(MG_EDEVICE, "FFT plan creation failed (" + std::to_string((int)r) + ")");
            break;
        }
        plans.emplace_back(kv.first, h);
    }
    if (out == MG_OK && e == hipSuccess) {
        int64_t toff = 0;
        for (auto &kv : L.by_m) {
            const int M = kv.first;
            for (int p : kv.second) {
                // one taper per plane keeps the screen's indexing plain (M
                // doubles each)
                double *c = taper + toff;
                hipLaunchKernelGGL(taper_kernel, dim3((M + 255) / 256), dim3(256), 0, stream, M,
                                   base_len, base_taps, c);
                const int64_t n = (int64_t)M * M;
                const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
                hipLaunchKernelGGL(screen_kernel, dim3(blocks), dim3(256), 0, stream, M, beta,
                                   plane_w[p], fov, (const double *)c, img + L.jobs[p].img_off);
                toff += M;
            }
        }
        for (auto &ph : plans) {
            const int p0 = L.by_m[ph.first].front();
            if (hipfftSetStream(ph.second, stream) != HIPFFT_SUCCESS ||
                hipfftExecZ2Z(ph.second, (hipfftDoubleComplex *)(img + L.jobs[p0].img_off),
                              (hipfftDoubleComplex *)(img + L.jobs[p0].img_off),
                              HIPFFT_FORWARD) != HIPFFT_SUCCESS) {
                out = set_error(MG_EDEVICE, "FFT execution failed");
                break;
            }
        }
    }
    if (out == MG_OK && e == hipSuccess) {
        int maxE = 0;
        for (auto &j : L.jobs) maxE = std::max(maxE, beta * j.S + 1);
        const dim3 g((unsigned)std::min(64, (maxE * maxE + 255) / 256), (unsigned)nplanes);
        hipLaunchKernelGGL(clear_max_kernel, dim3(1), dim3(1), 0, stream, mx);
        hipLaunchKernelGGL(maxabs_kernel, g, dim3(256), 0, stream, (const PlaneJob *)djobs, beta,
                           (const double2 *)img, mx);
        switch (out_dtype) {
        case MG_F16:
            hipLaunchKernelGGL(store_kernel<__half>, g, dim3(256), 0, stream,
                               (const PlaneJob *)djobs, beta, (const double2 *)img,
                               (const unsigned long long *)mx, (__half *)bank);
            break;
        case MG_BF16:
            hipLaunchKernelGGL(store_kernel<__hip_bfloat16>, g, dim3(256), 0, stream,
                               (const PlaneJob *)djobs, beta, (const double2 *)img,
                               (const unsigned long long *)mx, (__hip_bfloat16 *)bank);
            break;
        default:
            hipLaunchKernelGGL(store_kernel<float>, g, dim3(256), 0, stream,
                               (const PlaneJob *)djobs, beta, (const double2 *)img,
                               (const unsigned long long *)mx, (float *)bank);
            break;
        }
        e = hipGetLastError();
    }
    // the plans own work areas the transforms use: finish before freeing them
    const hipError_t es = hipStreamSynchronize(stream);
    for (auto &ph : plans) hipfftDestroy(ph.second);
    if (out != MG_OK) return out;
    if (e != hipSuccess || es != hipSuccess)
        return set_error(MG_EDEVICE, std::string("kernel bank: ") +
                                         hipGetErrorString(e != hipSuccess ? e : es));
    for (int p = 0; p < nplanes; ++p) plane_offset[p] = L.jobs[p].bank_off;
    return MG_OK;
}

}  // extern "C"
