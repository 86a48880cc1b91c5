// Image-plane steps around the hot path (the residual image of Eq. ResIm):
// the grid correction function of a separable kernel plane and the
// normalisation of F^dagger(grid) by the correction and the sum of weights.
// The Fourier transform itself runs in rocFFT, outside this library.
#include "lr_internal.h"
#include "lr_launch.h"

namespace lr {

// Element e of a table plane decoded to FP64 (f16 / bf16 divided by the
// plane's 2^e through its scale).
__device__ __forceinline__ double2 table_elem(const CFView &cf, int64_t e, float sc) {
    if (cf.storage == LR_F64) return ((const double2 *)cf.table)[e];
    if (cf.storage == LR_F32) {
        float2 v = ((const float2 *)cf.table)[e];
        return make_double2(v.x, v.y);
    }
    uint32_t b = ((const uint32_t *)cf.table)[e];
    float re, im;
    if (cf.storage == LR_F32_CF16) {
        _Float16 lo, hi;
        uint16_t l16 = (uint16_t)(b & 0xffffu), h16 = (uint16_t)(b >> 16);
        __builtin_memcpy(&lo, &l16, 2);
        __builtin_memcpy(&hi, &h16, 2);
        re = (float)lo;
        im = (float)hi;
    } else {
        re = __uint_as_float(b << 16);
        im = __uint_as_float(b & 0xffff0000u);
    }
    return make_double2((double)re * sc, (double)im * sc);
}

// Grid correction of a separable plane C[o_v][o_u][t_v][t_u] =
// c1[o_v][t_v] c1[o_u][t_u]: c1[o][t] is the o_v = 0, t_v = 0 row divided by
// sqrt(C at o = 0, t = 0), and gcf(xi) = (1/O) sum over o in [-O/2, O/2) and
// t of c1[o][t] exp(2 pi i (t - o/O) xi) at xi = (i - n/2) / n: the mean
// image-plane response of one sample over its possible offsets.
__global__ void k_gcf(CFView cf, int64_t plane_base, int32_t h, float sc, int32_t n,
                      double2 *out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int O = cf.O, S = 2 * h + 1, no = O + 1;
    const double xi = (double)(i - n / 2) / (double)n;
    // element of (o_v index, o_u index, t_v index, t_u index)
    auto at = [&](int ov, int ou, int tv, int tu) {
        return plane_base + (((int64_t)ov * no + ou) * S + tv) * S + tu;
    };
    const int mid = O / 2;
    const double2 c00 = table_elem(cf, at(mid, mid, h, h), sc);
    // sqrt of the (complex) centre value
    const double r = sqrt(hypot(c00.x, c00.y));
    const double ph = 0.5 * atan2(c00.y, c00.x);
    const double sr = r * cos(ph), si = r * sin(ph);
    const double den = sr * sr + si * si;
    double re = 0.0, im = 0.0;
    for (int oi = 0; oi < O; ++oi) {             // o = oi - O/2 in [-O/2, O/2)
        const double o = (double)(oi - mid);
        for (int ti = 0; ti < S; ++ti) {
            const double2 c = table_elem(cf, at(mid, oi, h, ti), sc);
            // c1 = c / sqrt(c00)
            const double c1r = (c.x * sr + c.y * si) / den;
            const double c1i = (c.y * sr - c.x * si) / den;
            double s, co;
            sincospi(2.0 * ((double)(ti - h) - o / O) * xi, &s, &co);
            re += c1r * co - c1i * s;
            im += c1r * s + c1i * co;
        }
    }
    out[i] = make_double2(re / O, im / O);
}

hipError_t launch_gcf(const CFView &cf, int64_t plane_base, int32_t h, float sc, int32_t n,
                      double2 *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gcf, dim3((n + 127) / 128), dim3(128), 0, s, cf, plane_base, h, sc, n,
                       out);
    return hipGetLastError();
}

// img[P][pol][iy][ix] (complex, the centred F^dagger of a grid) ->
// out = Re(img) / (gcf_x[ix] gcf_y[iy] sumwt[P][pol]).
template <typename T>
__global__ __launch_bounds__(256) void k_normalize(const T *img, const double *gx,
                                                   const double *gy, const double *sumwt,
                                                   int32_t nx, int32_t ny, int64_t n_planes,
                                                   T *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)nx * ny;
    if (i >= per * n_planes) return;
    const int64_t pl = i / per;
    const int64_t r = i - pl * per;
    const int iy = (int)(r / nx), ix = (int)(r - (int64_t)iy * nx);
    const double d = gx[ix] * gy[iy] * sumwt[pl];
    out[i] = (T)((double)img[2 * i] / d);
}

hipError_t launch_normalize(const void *img, const double *gx, const double *gy,
                            const double *sumwt, int32_t nx, int32_t ny, int64_t n_planes,
                            int precision, void *out, hipStream_t s) {
    const int64_t n = (int64_t)nx * ny * n_planes;
    if (n == 0) return hipSuccess;
    dim3 grd((unsigned)((n + 255) / 256)), blk(256);
    if (precision == LR_F64)
        hipLaunchKernelGGL(k_normalize<double>, grd, blk, 0, s, (const double *)img, gx, gy,
                           sumwt, nx, ny, n_planes, (double *)out);
    else
        hipLaunchKernelGGL(k_normalize<float>, grd, blk, 0, s, (const float *)img, gx, gy,
                           sumwt, nx, ny, n_planes, (float *)out);
    return hipGetLastError();
}

// As k_normalize, also divided by the weight image pb (same layout as
// out) where pb >= pb_min; 0 elsewhere.
template <typename T>
__global__ __launch_bounds__(256) void k_normalize_pb(const T *img, const double *gx,
                                                      const double *gy, const double *sumwt,
                                                      const double *pb, double pb_min,
                                                      int32_t nx, int32_t ny, int64_t n_planes,
                                                      T *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)nx * ny;
    if (i >= per * n_planes) return;
    const int64_t pl = i / per;
    const int64_t r = i - pl * per;
    const int iy = (int)(r / nx), ix = (int)(r - (int64_t)iy * nx);
    const double b = pb[i];
    out[i] = b >= pb_min ? (T)((double)img[2 * i] / (gx[ix] * gy[iy] * sumwt[pl] * b)) : (T)0;
}

hipError_t launch_normalize_pb(const void *img, const double *gx, const double *gy,
                               const double *sumwt, const double *pb, double pb_min,
                               int32_t nx, int32_t ny, int64_t n_planes, int precision,
                               void *out, hipStream_t s) {
    const int64_t n = (int64_t)nx * ny * n_planes;
    if (n == 0) return hipSuccess;
    dim3 grd((unsigned)((n + 255) / 256)), blk(256);
    if (precision == LR_F64)
        hipLaunchKernelGGL(k_normalize_pb<double>, grd, blk, 0, s, (const double *)img, gx, gy,
                           sumwt, pb, pb_min, nx, ny, n_planes, (double *)out);
    else
        hipLaunchKernelGGL(k_normalize_pb<float>, grd, blk, 0, s, (const float *)img, gx, gy,
                           sumwt, pb, pb_min, nx, ny, n_planes, (float *)out);
    return hipGetLastError();
}

}  // namespace lr
