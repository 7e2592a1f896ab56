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
//   the platform library's Z2Z forward FFT (one plan per size M and device,
//                  created on first use and kept for the process)
//   maxabs_kernel  largest |K| over every plane's kept samples
//   store_kernel   bank = K / max, converted to the output tap format, row
//                  (v offset) major.
// Plane parameters travel as kernel arguments (one launch per plane and
// step), so the call copies nothing from the host and does not synchronise.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
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

__global__ __launch_bounds__(256) void maxabs_kernel(int32_t M, int32_t E,
                                                     const double2 *__restrict__ buf,
                                                     unsigned long long *mx) {
    const int half = (E - 1) / 2;
    double best = 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < E * E; t += gridDim.x * blockDim.x) {
        const int ta = t / E, tb = t - ta * E;
        const double2 v = buf[kept_index(ta, tb, M, half)];
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
__global__ __launch_bounds__(256) void store_kernel(int32_t M, int32_t E,
                                                    const double2 *__restrict__ buf,
                                                    const unsigned long long *mx,
                                                    OutT *__restrict__ bank) {
    const int half = (E - 1) / 2;
    const double m = __longlong_as_double((long long)*mx);
    const double inv = m > 0.0 ? 1.0 / m : 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < E * E; t += gridDim.x * blockDim.x) {
        const int ta = t / E, tb = t - ta * E;
        const double2 v = buf[kept_index(ta, tb, M, half)];
        store_tap<OutT>(bank, t, v.x * inv, v.y * inv);
    }
}

// FFT plans by (device, M), kept for the life of the process.
std::mutex g_fft_mu;
std::map<std::pair<int, int>, hipfftHandle> g_fft;

hipfftResult fft_plan(int M, hipfftHandle *h) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HIPFFT_INTERNAL_ERROR;
    std::lock_guard<std::mutex> lk(g_fft_mu);
    auto it = g_fft.find({dev, M});
    if (it != g_fft.end()) {
        *h = it->second;
        return HIPFFT_SUCCESS;
    }
    const hipfftResult r = hipfftPlan2d(h, M, M, HIPFFT_Z2Z);
    if (r == HIPFFT_SUCCESS) g_fft[{dev, M}] = *h;
    return r;
}

struct Layout {
    std::vector<PlaneJob> jobs;
    int64_t bank_elems = 0;
    int64_t img_elems = 0;
    int64_t taper_elems = 0;
    size_t bytes = 0;
    size_t off_img = 0, off_taper = 0, off_max = 0;
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
        PlaneJob &j = L.jobs[p];
        j.S = S;
        j.M = 2 * beta * S;
        j.bank_off = L.bank_elems;
        L.bank_elems += (int64_t)(beta * S + 1) * (beta * S + 1);
        j.img_off = L.img_elems;
        L.img_elems += (int64_t)j.M * j.M;
        L.taper_elems += j.M;
    }
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t at = off;
        off += arena_round(b);
        return at;
    };
    L.off_img = take(sizeof(double2) * (size_t)L.img_elems);
    L.off_taper = take(sizeof(double) * (size_t)L.taper_elems);
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
    unsigned long long *mx = reinterpret_cast<unsigned long long *>(ws + L.off_max);

    hipLaunchKernelGGL(clear_max_kernel, dim3(1), dim3(1), 0, stream, mx);
    int64_t toff = 0;
    for (int p = 0; p < nplanes; ++p) {
        const PlaneJob &j = L.jobs[p];
        const int M = j.M, E = beta * j.S + 1;
        double *c = taper + toff;
        toff += M;
        double2 *buf = img + j.img_off;
        hipLaunchKernelGGL(taper_kernel, dim3((M + 255) / 256), dim3(256), 0, stream, M, base_len,
                           base_taps, c);
        const int64_t n = (int64_t)M * M;
        hipLaunchKernelGGL(screen_kernel, dim3((int)std::min<int64_t>((n + 255) / 256, 4096)),
                           dim3(256), 0, stream, M, beta, plane_w[p], fov, (const double *)c, buf);
        hipfftHandle h = 0;
        hipfftResult r = fft_plan(M, &h);
        if (r == HIPFFT_SUCCESS) {
            // the plan is shared: its stream is set and the transform queued
            // under the lock
            std::lock_guard<std::mutex> lk(g_fft_mu);
            r = hipfftSetStream(h, stream);
            if (r == HIPFFT_SUCCESS)
                r = hipfftExecZ2Z(h, (hipfftDoubleComplex *)buf, (hipfftDoubleComplex *)buf,
                                  HIPFFT_FORWARD);
        }
        if (r != HIPFFT_SUCCESS)
            return set_error(MG_EDEVICE, "FFT failed (" + std::to_string((int)r) + ")");
        hipLaunchKernelGGL(maxabs_kernel, dim3((unsigned)std::min(64, (E * E + 255) / 256)),
                           dim3(256), 0, stream, M, E, (const double2 *)buf, mx);
    }
    for (int p = 0; p < nplanes; ++p) {
        const PlaneJob &j = L.jobs[p];
        const int M = j.M, E = beta * j.S + 1;
        const double2 *buf = img + j.img_off;
        const dim3 g((unsigned)std::min(256, (E * E + 255) / 256));
        switch (out_dtype) {
        case MG_F16:
            hipLaunchKernelGGL(store_kernel<__half>, g, dim3(256), 0, stream, M, E, buf,
                               (const unsigned long long *)mx,
                               (__half *)bank + 2 * j.bank_off);
            break;
        case MG_BF16:
            hipLaunchKernelGGL(store_kernel<__hip_bfloat16>, g, dim3(256), 0, stream, M, E, buf,
                               (const unsigned long long *)mx,
                               (__hip_bfloat16 *)bank + 2 * j.bank_off);
            break;
        default:
            hipLaunchKernelGGL(store_kernel<float>, g, dim3(256), 0, stream, M, E, buf,
                               (const unsigned long long *)mx, (float *)bank + 2 * j.bank_off);
            break;
        }
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(MG_EDEVICE, std::string("kernel bank: ") + hipGetErrorString(e));
    for (int p = 0; p < nplanes; ++p) plane_offset[p] = L.jobs[p].bank_off;
    return MG_OK;
}

}  // extern "C"
