// Hogbom minor cycle (the ModelUpdate step of the imaging section): loop
// gain, threshold exit, one image plane.
//
// One launch per iteration.  Each launch subtracts gain x peak x PSF (its
// centre (ny/2, nx/2) on the peak found by the previous launch) from the
// residual, adds gain x peak to the model, and finds the next peak in the
// same pass: every workgroup reduces its pixels to (|r|, index) and the
// last workgroup to finish (a global counter) reduces those partials and
// writes the peak, the iteration count and the stop flag into a small
// state record that the next launch reads.  Launch 0 only searches.  Once
// the stop flag is set later launches return at once, so a caller may
// enqueue the whole budget without waiting.  Ties go to the lowest index.
#include "lr_internal.h"
#include "lr_launch.h"

namespace lr {

struct HogbomState {
    double peak;          // signed value at the peak
    int64_t idx;          // its row-major index
    int32_t iter;         // subtractions done
    int32_t stop;
    uint32_t arrived;     // workgroups finished in this launch
    int32_t pad;
};

struct Cand {
    double a;             // |value|
    double v;             // value
    int64_t i;            // index (-1: none)
};

__device__ __forceinline__ bool better(const Cand &x, const Cand &y) {
    return x.a > y.a || (x.a == y.a && x.i >= 0 && (y.i < 0 || x.i < y.i));
}

__device__ __forceinline__ Cand shfl_cand(const Cand &c, int off) {
    Cand o;
    o.a = __shfl_xor(c.a, off);
    o.v = __shfl_xor(c.v, off);
    o.i = (int64_t)__shfl_xor((long long)c.i, off);
    return o;
}

// Best candidate of the workgroup, returned in thread 0.
__device__ Cand block_best(Cand c) {
    __shared__ Cand part[1024 / 64];
    for (int off = 32; off > 0; off >>= 1) {
        Cand o = shfl_cand(c, off);
        if (better(o, c)) c = o;
    }
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if ((threadIdx.x & 63) == 0) part[w] = c;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 1; k < nw; ++k)
            if (better(part[k], c)) c = part[k];
    return c;
}

template <typename T>
__global__ __launch_bounds__(256) void k_hogbom(T *res, const T *psf, T *model, int32_t nx,
                                               int32_t ny, double gain, double threshold,
                                               int32_t niter, int32_t search_only,
                                               HogbomState *st, Cand *partials) {
    if (st->stop) return;
    const int64_t n = (int64_t)nx * ny;
    const bool sub = !search_only;
    // the scale is rounded to T before use, in the precision of the image
    const T c = sub ? (T)(gain * st->peak) : (T)0;
    const int64_t pidx = st->idx;
    const int py = (int)(pidx / nx), px = (int)(pidx - (int64_t)py * nx);
    const int cy = ny / 2, cx = nx / 2;
    if (sub && blockIdx.x == 0 && threadIdx.x == 0) model[pidx] += c;
    Cand best{-1.0, 0.0, -1};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        T r = res[i];
        if (sub) {
            const int y = (int)(i / nx), x = (int)(i - (int64_t)y * nx);
            const int sy = y - py + cy, sx = x - px + cx;
            if ((unsigned)sy < (unsigned)ny && (unsigned)sx < (unsigned)nx) {
                r = r - c * psf[(int64_t)sy * nx + sx];
                res[i] = r;
            }
        }
        const double a = fabs((double)r);
        if (a > best.a) best = Cand{a, (double)r, i};   // i increases: first wins ties
    }
    best = block_best(best);
    __shared__ bool last;
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = best;
        __threadfence();
        last = atomicAdd(&st->arrived, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    // the last workgroup to arrive reduces the partials
    __threadfence();
    Cand g{-1.0, 0.0, -1};
    for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) {
        Cand p = partials[b];
        if (better(p, g)) g = p;
    }
    g = block_best(g);
    if (threadIdx.x == 0) {
        const int32_t it = st->iter + (sub ? 1 : 0);
        st->iter = it;
        st->peak = g.v;
        st->idx = g.i < 0 ? 0 : g.i;
        st->stop = (g.i < 0 || g.a < threshold || it >= niter) ? 1 : 0;
        st->arrived = 0;
    }
}

__global__ void k_hogbom_reset(HogbomState *st) {
    if (threadIdx.x == 0) {
        st->peak = 0.0;
        st->idx = 0;
        st->iter = 0;
        st->stop = 0;
        st->arrived = 0;
        st->pad = 0;
    }
}

size_t hogbom_work_bytes(int32_t nx, int32_t ny) {
    (void)nx;
    (void)ny;
    return 256 + sizeof(Cand) * kHogbomBlocks;
}

hipError_t launch_hogbom(void *res, const void *psf, void *model, int32_t nx, int32_t ny,
                         int precision, double gain, double threshold, int32_t niter,
                         void *work, int32_t *iters, hipStream_t s) {
    HogbomState *st = (HogbomState *)work;
    Cand *part = (Cand *)((char *)work + 256);
    const int64_t n = (int64_t)nx * ny;
    const unsigned blocks = (unsigned)std::min<int64_t>(kHogbomBlocks, (n + 255) / 256);
    hipLaunchKernelGGL(k_hogbom_reset, dim3(1), dim3(64), 0, s, st);
    for (int32_t k = 0; k <= niter; ++k) {
        if (precision == LR_F64)
            hipLaunchKernelGGL(k_hogbom<double>, dim3(blocks), dim3(256), 0, s, (double *)res,
                               (const double *)psf, (double *)model, nx, ny, gain, threshold,
                               niter, k == 0 ? 1 : 0, st, part);
        else
            hipLaunchKernelGGL(k_hogbom<float>, dim3(blocks), dim3(256), 0, s, (float *)res,
                               (const float *)psf, (float *)model, nx, ny, gain, threshold,
                               niter, k == 0 ? 1 : 0, st, part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    HogbomState h;
    hipError_t e = hipMemcpyAsync(&h, st, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) *iters = h.iter;
    return e;
}

}  // namespace lr
