// Change of phase centre for mosaic imaging (the mosaic rows of the
// imaging-mode table; Eq. CIJ): every sample of a row of field f is
// multiplied by exp(sign 2 pi i (u l_f + v m_f)), u and v in wavelengths,
// with the argument formed in FP64 and reduced modulo 1 before the sine and
// cosine (sign -1 moves the data from the field's phase centre to the joint
// image centre, +1 back).  One thread per (row, channel) pair; the channel
// scales nu / c travel in the kernel argument, 64 channels per launch.
#include "lr_internal.h"
#include "lr_launch.h"

namespace lr {

constexpr int kRephaseChan = 64;

struct RephaseArgs {
    void *vis;
    const double *uvw;
    const int32_t *field;
    const double *field_dlm;
    int64_t nrow;
    int32_t nchan, npol, nfield, c0, nc;
    double sign;
    double s[kRephaseChan];     // nu / c of channels c0 .. c0 + nc - 1
};

template <typename T>
__global__ __launch_bounds__(256) void k_rephase(RephaseArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.nrow * a.nc) return;
    const int64_t r = t / a.nc;
    const int cl = (int)(t - r * a.nc);
    const int f = a.field[r];
    if (f < 0 || f >= a.nfield) return;          // rows outside every field: unchanged
    const double u = a.uvw[3 * r] * a.s[cl], v = a.uvw[3 * r + 1] * a.s[cl];
    double x = u * a.field_dlm[2 * f] + v * a.field_dlm[2 * f + 1];
    x = x - rint(x);
    double sn, cs;
    sincospi(a.sign * 2.0 * x, &sn, &cs);
    T *p = (T *)a.vis + 2 * ((r * a.nchan + a.c0 + cl) * a.npol);
    for (int k = 0; k < a.npol; ++k) {
        const double re = (double)p[2 * k], im = (double)p[2 * k + 1];
        p[2 * k] = (T)(re * cs - im * sn);
        p[2 * k + 1] = (T)(re * sn + im * cs);
    }
}

hipError_t launch_rephase(void *vis, const double *uvw, const double *freq_hz,
                          const int32_t *field, const double *field_dlm, int64_t nrow,
                          int32_t nchan, int32_t npol, int32_t nfield, int precision,
                          int32_t direction, hipStream_t s) {
    for (int32_t c0 = 0; c0 < nchan; c0 += kRephaseChan) {
        RephaseArgs a;
        a.vis = vis;
        a.uvw = uvw;
        a.field = field;
        a.field_dlm = field_dlm;
        a.nrow = nrow;
        a.nchan = nchan;
        a.npol = npol;
        a.nfield = nfield;
        a.c0 = c0;
        a.nc = std::min<int32_t>(kRephaseChan, nchan - c0);
        a.sign = direction < 0 ? -1.0 : 1.0;
        for (int i = 0; i < a.nc; ++i) a.s[i] = freq_hz[c0 + i] / kCLight;
        const int64_t n = nrow * a.nc;
        if (n == 0) continue;
        dim3 grd((unsigned)((n + 255) / 256)), blk(256);
        if (precision == LR_F64) hipLaunchKernelGGL(k_rephase<double>, grd, blk, 0, s, a);
        else hipLaunchKernelGGL(k_rephase<float>, grd, blk, 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace lr
