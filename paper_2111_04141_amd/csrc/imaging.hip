// Imaging chain: origin shift, inverse FFT and the Correction Step.
//
// The grids have their origin at the centre (cell n/2 is u = 0).  For even
// sizes the centred unnormalised inverse transform
//     I[y, x] = sum_k G[kv, ku] exp(+j2pi ((ku - nx/2)(x - nx/2)/nx + ...))
// is (-1)^(x + y + nx/2 + ny/2) times the plain inverse FFT of
// (-1)^(ku + kv) G, so the origin shifts are two sign flips fused into the
// kernels around the FFT (the batched C2C transform of the platform library,
// one per polarisation).  The Correction Step (Section 2.4.5, corrector h_co;
// Section 2.4.4 for Hybrid Gridding, with the pruning kernel's corrector
// along v) multiplies by separable corrector vectors, computed on the device
// from the kernel tables (corrector_kernel):
//     h(l) = 1 / ( (1/P) sum_e T[e] cos(2pi ((e - E/2)/beta) l) sinc(l/beta) ),
// l = (i - n/2)/n, for a symmetric table T of E + 1 values whose entry e lies
// (e - E/2)/beta cells from the centre, averaged over its P sub-cell phases.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cmath>
#include <new>
#include <string>

#include "internal.h"

struct mg_imager {
    hipfftHandle plan = 0;
    int32_t npol = 0, nx = 0, ny = 0;
};

struct mg_wstack_imager {
    hipfftHandle plan = 0;
    int32_t npol = 0, layers = 0, nx = 0, ny = 0;
};

namespace mg {
namespace {

__global__ __launch_bounds__(256) void corrector_kernel(int32_t n, int32_t beta, int32_t ntab,
                                                        int32_t phases, int32_t nn_sinc,
                                                        const float *__restrict__ table,
                                                        float *__restrict__ corr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double l = (double)(i - n / 2) / (double)n;
    const double half = 0.5 * (double)(ntab - 1);
    const double two_pi = 6.283185307179586476925286766559;
    double s = 0.0;
    for (int e = 0; e < ntab; ++e)
        s += (double)table[e] * cos(two_pi * (((double)e - half) / (double)beta) * l);
    s /= (double)phases;
    if (nn_sinc) {
        const double a = 3.14159265358979323846264338328 * l / (double)beta;
        s *= (a == 0.0) ? 1.0 : sin(a) / a;
    }
    corr[i] = (float)(1.0 / s);
}

// work[p][y][x] = (-1)^(x + y) grid[p][y][x]
__global__ __launch_bounds__(256) void shift_in_kernel(const float2 *__restrict__ grid,
                                                       float2 *__restrict__ work, int32_t nx,
                                                       int64_t total) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = k / nx;
        const int x = (int)(k - row * nx);
        float2 g = grid[k];
        if ((x + row) & 1) {
            g.x = -g.x;
            g.y = -g.y;
        }
        work[k] = g;
    }
}

// image[p][y][x] = (-1)^(x + y0 + y + nx/2 + ny/2) corr_x[x] corr_y[y]
//                  work[p][y0 + y][x], y < out_ny
__global__ __launch_bounds__(256) void correct_out_kernel(const float2 *__restrict__ work,
                                                          float2 *__restrict__ image, int32_t nx,
                                                          int32_t ny, int32_t y0, int32_t out_ny,
                                                          int32_t npol,
                                                          const float *__restrict__ cx,
                                                          const float *__restrict__ cy) {
    const int64_t total = (int64_t)npol * out_ny * nx;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t prow = k / nx;
        const int x = (int)(k - prow * nx);
        const int p = (int)(prow / out_ny);
        const int y = (int)(prow - (int64_t)p * out_ny);
        float2 v = work[((int64_t)p * ny + y0 + y) * nx + x];
        float f = cx[x] * cy[y];
        if ((x + y0 + y + nx / 2 + ny / 2) & 1) f = -f;
        v.x *= f;
        v.y *= f;
        image[k] = v;
    }
}

// W-stacking: image[p][y][x] = (-1)^(x + y + nx/2 + ny/2) cx[x] cy[y]
//   sum_j work[p][j][y][x] gbar_{w_j}(l_x, m_y),
// gbar_w = exp(+j2pi w (sqrt(1 - l^2 - m^2) - 1)), w_j = (j - (L-1)/2) dw,
// l_x = (x - nx/2)/nx fov_x, m_y = (y - ny/2)/ny fov_y.  n - 1 is formed as
// -r^2 / (1 + sqrt(1 - r^2)) (no cancellation) and each phase, in cycles, is
// reduced to (-1/2, 1/2] in FP64 before the FP32 sine and cosine.
__global__ __launch_bounds__(256) void wstack_combine_kernel(
    const float2 *__restrict__ work, float2 *__restrict__ image, int32_t nx, int32_t ny,
    int32_t npol, int32_t layers, double dw, double fov_x, double fov_y,
    const float *__restrict__ cx, const float *__restrict__ cy) {
    const int64_t plane = (int64_t)ny * nx;
    const int64_t total = (int64_t)npol * plane;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(k / plane);
        const int64_t yx = k - (int64_t)p * plane;
        const int y = (int)(yx / nx);
        const int x = (int)(yx - (int64_t)y * nx);
        const double l = (double)(x - nx / 2) / (double)nx * fov_x;
        const double m = (double)(y - ny / 2) / (double)ny * fov_y;
        const double r2 = l * l + m * m;
        const double nm1 = r2 < 1.0 ? -r2 / (1.0 + sqrt(1.0 - r2)) : -1.0;
        float sr = 0.0f, si = 0.0f;
        const float2 *src = work + (int64_t)p * layers * plane + yx;
        for (int j = 0; j < layers; ++j) {
            const double wj = ((double)j - 0.5 * (double)(layers - 1)) * dw;
            double cyc = wj * nm1;
            cyc -= rint(cyc);
            float sn, cs;
            sincosf(6.283185307179586f * (float)cyc, &sn, &cs);
            const float2 v = src[(int64_t)j * plane];
            sr += v.x * cs - v.y * sn;
            si += v.x * sn + v.y * cs;
        }
        float f = cx[x] * cy[y];
        if ((x + y + nx / 2 + ny / 2) & 1) f = -f;
        image[k] = make_float2(sr * f, si * f);
    }
}

int blocks_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

}  // namespace
}  // namespace mg

using namespace mg;

extern "C" {

mg_status mg_corrector(int32_t n, int32_t beta, int32_t table_len, int32_t phases,
                       int32_t nn_sinc, const float *table, float *corr, hipStream_t stream) {
    if (n < 1 || beta < 1 || table_len < 1 || phases < 1 || !table || !corr)
        return set_error(MG_EINVAL, "bad corrector arguments");
    hipLaunchKernelGGL(corrector_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       n, beta, table_len, phases, nn_sinc, table, corr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(MG_EDEVICE, std::string("corrector: ") + hipGetErrorString(e));
    return MG_OK;
}

mg_status mg_imager_create(mg_imager **im, int32_t npol, int32_t nx, int32_t ny) {
    if (!im) return set_error(MG_EINVAL, "null imager output");
    *im = nullptr;
    if (npol < 1 || npol > 4 || nx < 2 || ny < 2 || (nx & 1) || (ny & 1))
        return set_error(MG_EINVAL, "imager sizes must be even, npol 1..4");
    mg_imager *p = new (std::nothrow) mg_imager;
    if (!p) return set_error(MG_ENOMEM, "host allocation failed");
    p->npol = npol;
    p->nx = nx;
    p->ny = ny;
    int dims[2] = {ny, nx};
    const int dist = ny * nx;
    const hipfftResult r = hipfftPlanMany(&p->plan, 2, dims, nullptr, 1, dist, nullptr, 1, dist,
                                          HIPFFT_C2C, npol);
    if (r != HIPFFT_SUCCESS) {
        delete p;
        return set_error(MG_EDEVICE, "FFT plan creation failed (" + std::to_string((int)r) + ")");
    }
    *im = p;
    return MG_OK;
}

mg_status mg_imager_exec(mg_imager *im, const void *grid, void *work, void *image,
                         const float *corr_x, const float *corr_y, int32_t y0, int32_t out_ny,
                         hipStream_t stream) {
    if (!im || !grid || !work || !image || !corr_x || !corr_y)
        return set_error(MG_EINVAL, "null argument");
    if (y0 < 0 || out_ny < 1 || y0 + out_ny > im->ny)
        return set_error(MG_EINVAL, "rows out of range");
    if (work == image && !(y0 == 0 && out_ny == im->ny))
        return set_error(MG_EINVAL, "a cropped image needs its own buffer");
    const int64_t total = (int64_t)im->npol * im->ny * im->nx;
    hipLaunchKernelGGL(shift_in_kernel, dim3(blocks_for(total)), dim3(256), 0, stream,
                       (const float2 *)grid, (float2 *)work, im->nx, total);
    if (hipfftSetStream(im->plan, stream) != HIPFFT_SUCCESS)
        return set_error(MG_EDEVICE, "FFT stream");
    const hipfftResult r = hipfftExecC2C(im->plan, (hipfftComplex *)work, (hipfftComplex *)work,
                                         HIPFFT_BACKWARD);
    if (r != HIPFFT_SUCCESS)
        return set_error(MG_EDEVICE, "FFT execution failed (" + std::to_string((int)r) + ")");
    hipLaunchKernelGGL(correct_out_kernel,
                       dim3(blocks_for((int64_t)im->npol * out_ny * im->nx)), dim3(256), 0, stream,
                       (const float2 *)work, (float2 *)image, im->nx, im->ny, y0, out_ny,
                       im->npol, corr_x, corr_y);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(MG_EDEVICE, std::string("imaging kernels: ") + hipGetErrorString(e));
    return MG_OK;
}

mg_status mg_imager_destroy(mg_imager *im) {
    if (!im) return MG_OK;
    if (im->plan) hipfftDestroy(im->plan);
    delete im;
    return MG_OK;
}

mg_status mg_wstack_imager_create(mg_wstack_imager **im, int32_t npol, int32_t layers,
                                  int32_t nx, int32_t ny) {
    if (!im) return set_error(MG_EINVAL, "null imager output");
    *im = nullptr;
    if (npol < 1 || npol > 4 || layers < 1 || layers > kMaxPlanes || nx < 2 || ny < 2 ||
        (nx & 1) || (ny & 1))
        return set_error(MG_EINVAL, "imager sizes must be even, npol 1..4, layers 1..128");
    mg_wstack_imager *p = new (std::nothrow) mg_wstack_imager;
    if (!p) return set_error(MG_ENOMEM, "host allocation failed");
    p->npol = npol;
    p->layers = layers;
    p->nx = nx;
    p->ny = ny;
    int dims[2] = {ny, nx};
    const int dist = ny * nx;
    const hipfftResult r = hipfftPlanMany(&p->plan, 2, dims, nullptr, 1, dist, nullptr, 1, dist,
                                          HIPFFT_C2C, npol * layers);
    if (r != HIPFFT_SUCCESS) {
        delete p;
        return set_error(MG_EDEVICE, "FFT plan creation failed (" + std::to_string((int)r) + ")");
    }
    *im = p;
    return MG_OK;
}

mg_status mg_wstack_imager_exec(mg_wstack_imager *im, const void *grids, void *work, void *image,
                                const float *corr_x, const float *corr_y, double fov_x,
                                double fov_y, double dw, hipStream_t stream) {
    if (!im || !grids || !work || !image || !corr_x || !corr_y)
        return set_error(MG_EINVAL, "null argument");
    if (!std::isfinite(fov_x) || !std::isfinite(fov_y) || !std::isfinite(dw))
        return set_error(MG_EINVAL, "fov and dw must be finite");
    if (work == image) return set_error(MG_EINVAL, "the image needs its own buffer");
    const int64_t total = (int64_t)im->npol * im->layers * im->ny * im->nx;
    hipLaunchKernelGGL(shift_in_kernel, dim3(blocks_for(total)), dim3(256), 0, stream,
                       (const float2 *)grids, (float2 *)work, im->nx, total);
    if (hipfftSetStream(im->plan, stream) != HIPFFT_SUCCESS)
        return set_error(MG_EDEVICE, "FFT stream");
    const hipfftResult r = hipfftExecC2C(im->plan, (hipfftComplex *)work, (hipfftComplex *)work,
                                         HIPFFT_BACKWARD);
    if (r != HIPFFT_SUCCESS)
        return set_error(MG_EDEVICE, "FFT execution failed (" + std::to_string((int)r) + ")");
    hipLaunchKernelGGL(wstack_combine_kernel,
                       dim3(blocks_for((int64_t)im->npol * im->ny * im->nx)), dim3(256), 0, stream,
                       (const float2 *)work, (float2 *)image, im->nx, im->ny, im->npol,
                       im->layers, dw, fov_x, fov_y, corr_x, corr_y);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(MG_EDEVICE, std::string("W-stacking kernels: ") + hipGetErrorString(e));
    return MG_OK;
}

mg_status mg_wstack_imager_destroy(mg_wstack_imager *im) {
    if (!im) return MG_OK;
    if (im->plan) hipfftDestroy(im->plan);
    delete im;
    return MG_OK;
}

}  // extern "C"
