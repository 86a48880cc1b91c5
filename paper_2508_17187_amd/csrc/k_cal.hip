// Diagonal G-Jones calibration (calibration section): the ratio averages of
// Eq. VAvg (PreSolvePrep) and the damped fixed-point solve of Eqs.
// CalUpdateDir / CalUpdateModel with the max-change exit (ExitCriteria).
//
// vavg      one thread per (column, block of steps): pair c + m L is step m
//           of column c (L = rows per step x channels, so a column is one
//           channel of one row slot of a dump); the thread keeps FP64 sums
//           W V conj(M) and W |M|^2 per parallel hand in registers while the
//           (interval, baseline) bin stays the same and adds them to the bin
//           with FP64 atomics when it changes.  Any rows-per-step value
//           gives the same sums; the row period of time-major data keeps
//           one baseline per column, so a thread flushes once per interval.
// finalize  one thread per antenna pair i < j: both orientations summed,
//           X = sum / weight written to (i, j) and its conjugate to (j, i).
// solve     one workgroup per problem (interval, hand): gains in LDS, the
//           update direction of every antenna from the same iterate, a
//           block maximum of the change for the exit test.
#include "lr_internal.h"
#include "lr_launch.h"

namespace lr {

struct VavgArgs {
    const void *obs, *mod, *weight;
    const int32_t *ant1, *ant2, *row_sol, *chan_sol;
    int64_t nrow;
    int32_t nchan, npol, nant, n_tsol, n_fsol, npar;
    int32_t rows_per_step, steps_per_thread;
    int64_t L, n_cols_blocks;
    double *X;       // complex [n_tsol][n_fsol][npar][nant][nant], zeroed: sums
    double *w;       // [n_tsol][n_fsol][npar][nant][nant], zeroed: sums
};

// parallel hands: XX, YY of four correlations; both of two; the one of one
__device__ __forceinline__ int hand(int npol, int q) { return npol == 4 ? 3 * q : q; }

template <typename T, int NPAR>
__global__ __launch_bounds__(256) void k_cal_vavg(VavgArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = t % a.L;
    const int64_t blk = t / a.L;
    // threads past the work stay (idle) for the wave-wide flushes
    const bool live = blk < a.n_cols_blocks;
    const int ch = (int)(c % a.nchan);
    const int64_t slot = c / a.nchan;
    // lanes of a channel outside every interval stay for the wave-wide
    // flushes but never hold a bin
    const int fs0 = a.chan_sol[ch];
    const bool chan_ok = fs0 >= 0 && fs0 < a.n_fsol;
    const int fs = chan_ok ? fs0 : 0;
    const int64_t m0 = blk * a.steps_per_thread;
    const int64_t nn = (int64_t)a.nant * a.nant;
    int64_t bin = -1;                       // bin of hand 0; hand q adds q * nn
    double nr[NPAR], ni[NPAR], dw[NPAR];
    for (int q = 0; q < NPAR; ++q) nr[q] = ni[q] = dw[q] = 0.0;
    const int lane = threadIdx.x & 63;
    // Lanes whose bin closes add their sums to it.  Neighbouring lanes (the
    // channels of one frequency interval of one baseline) usually close the
    // same bin at the same step: a segmented sum over runs of equal bins
    // leaves one atomic per run.  Every lane of the wavefront takes part.
    auto flush = [&](bool closing) {
        // runs of lanes closing the same bin; every other lane a run of its
        // own (a bin closed by two separate runs gets one atomic per run)
        const int64_t key = closing && bin >= 0 ? bin : -1 - (int64_t)lane;
        const int64_t kp = __shfl_up(key, 1);
        const uint64_t heads = __ballot(lane == 0 || kp != key);
        const int seg = __popcll(heads & ((2ull << lane) - 1));
        for (int off = 1; off < 64; off <<= 1) {
            const int so = __shfl_up(seg, off);
            const bool take = lane >= off && so == seg;
            for (int q = 0; q < NPAR; ++q) {
                const double r = __shfl_up(nr[q], off), im = __shfl_up(ni[q], off),
                             d = __shfl_up(dw[q], off);
                if (take && closing) {
                    nr[q] += r;
                    ni[q] += im;
                    dw[q] += d;
                }
            }
        }
        const int sn = __shfl_down(seg, 1);
        const bool last = lane == 63 || sn != seg;
        if (closing) {
            for (int q = 0; q < NPAR; ++q) {
                if (last && bin >= 0 && dw[q] != 0.0) {
                    const int64_t b = bin + q * nn;
                    atomicAdd(&a.X[2 * b], nr[q]);
                    atomicAdd(&a.X[2 * b + 1], ni[q]);
                    atomicAdd(&a.w[b], dw[q]);
                }
                nr[q] = ni[q] = dw[q] = 0.0;
            }
        }
    };
    for (int s = 0; s < a.steps_per_thread; ++s) {
        const int64_t row = slot + (m0 + s) * a.rows_per_step;
        const bool in = live && chan_ok && row < a.nrow;
        int i = 0, j = 0, ts = -1;
        if (in) {
            i = a.ant1[row];
            j = a.ant2[row];
            ts = a.row_sol[row];
        }
        // autocorrelations, rows outside every interval and ids out of range
        const bool use = in && i != j && ts >= 0 && ts < a.n_tsol &&
                         (unsigned)i < (unsigned)a.nant && (unsigned)j < (unsigned)a.nant;
        const int64_t b =
            use ? ((((int64_t)ts * a.n_fsol + fs) * NPAR) * a.nant + i) * a.nant + j : bin;
        const bool closing = use && b != bin;
        if (__any(closing)) flush(closing);
        if (closing) bin = b;
        if (!use) continue;
        const int64_t e = (row * a.nchan + ch) * a.npol;
        const T *ov = (const T *)a.obs + 2 * e;
        const T *mv = (const T *)a.mod + 2 * e;
        const T *wv = a.weight ? (const T *)a.weight + e : nullptr;
        for (int q = 0; q < NPAR; ++q) {
            const int p = hand(a.npol, q);
            const double W = wv ? (double)wv[p] : 1.0;
            const double mr = (double)mv[2 * p], mi = (double)mv[2 * p + 1];
            if (!(W > 0.0) || (mr == 0.0 && mi == 0.0)) continue;
            const double vr = (double)ov[2 * p], vi = (double)ov[2 * p + 1];
            // W V conj(M) and W |M|^2
            nr[q] += W * (vr * mr + vi * mi);
            ni[q] += W * (vi * mr - vr * mi);
            dw[q] += W * (mr * mr + mi * mi);
        }
    }
    flush(bin >= 0);
}

__global__ void k_cal_finalize(double *X, double *w, int32_t nant, int64_t n_mat) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nn = (int64_t)nant * nant;
    if (t >= n_mat * nn) return;
    const int64_t mat = t / nn;
    const int i = (int)((t % nn) / nant), j = (int)(t % nant);
    if (i > j) return;
    double *Xm = X + 2 * mat * nn;
    double *wm = w + mat * nn;
    const int64_t ij = (int64_t)i * nant + j, ji = (int64_t)j * nant + i;
    if (i == j) {
        Xm[2 * ij] = Xm[2 * ij + 1] = 0.0;
        wm[ij] = 0.0;
        return;
    }
    // (i, j) holds sum W V conj(M) of rows i-j; (j, i) that of rows j-i,
    // whose conjugate belongs to i-j
    const double sr = Xm[2 * ij] + Xm[2 * ji], si = Xm[2 * ij + 1] - Xm[2 * ji + 1];
    const double sw = wm[ij] + wm[ji];
    const double xr = sw > 0.0 ? sr / sw : 0.0, xi = sw > 0.0 ? si / sw : 0.0;
    Xm[2 * ij] = xr;
    Xm[2 * ij + 1] = xi;
    Xm[2 * ji] = xr;
    Xm[2 * ji + 1] = -xi;
    wm[ij] = sw;
    wm[ji] = sw;
}

__global__ void k_cal_zero(double *p, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0;
}

hipError_t launch_cal_vavg(const CalVavg &c, hipStream_t s) {
    const int npar = c.npol == 1 ? 1 : 2;
    const int64_t n_mat = (int64_t)c.n_tsol * c.n_fsol * npar;
    const int64_t nn = (int64_t)c.nant * c.nant;
    const int64_t nx = 2 * n_mat * nn, nw = n_mat * nn;
    hipLaunchKernelGGL(k_cal_zero, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, s, c.X, nx);
    hipLaunchKernelGGL(k_cal_zero, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, c.w, nw);
    if (c.nrow > 0 && c.nchan > 0) {
        VavgArgs a;
        a.obs = c.obs;
        a.mod = c.mod;
        a.weight = c.weight;
        a.ant1 = c.ant1;
        a.ant2 = c.ant2;
        a.row_sol = c.row_sol;
        a.chan_sol = c.chan_sol;
        a.nrow = c.nrow;
        a.nchan = c.nchan;
        a.npol = c.npol;
        a.nant = c.nant;
        a.n_tsol = c.n_tsol;
        a.n_fsol = c.n_fsol;
        a.npar = npar;
        a.rows_per_step = c.rows_per_step;
        a.steps_per_thread = 16;
        a.L = (int64_t)c.rows_per_step * c.nchan;
        const int64_t steps = (c.nrow + c.rows_per_step - 1) / c.rows_per_step;
        a.n_cols_blocks = (steps + a.steps_per_thread - 1) / a.steps_per_thread;
        a.X = c.X;
        a.w = c.w;
        const int64_t threads = a.L * a.n_cols_blocks;
        dim3 grd((unsigned)((threads + 255) / 256)), blk(256);
        const bool f64 = c.precision == LR_F64;
        if (npar == 1) {
            if (f64) hipLaunchKernelGGL((k_cal_vavg<double, 1>), grd, blk, 0, s, a);
            else hipLaunchKernelGGL((k_cal_vavg<float, 1>), grd, blk, 0, s, a);
        } else {
            if (f64) hipLaunchKernelGGL((k_cal_vavg<double, 2>), grd, blk, 0, s, a);
            else hipLaunchKernelGGL((k_cal_vavg<float, 2>), grd, blk, 0, s, a);
        }
    }
    const int64_t n = n_mat * nn;
    if (n > 0)
        hipLaunchKernelGGL(k_cal_finalize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           c.X, c.w, c.nant, n_mat);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_max(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double r = red[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) r = fmax(r, red[k]);
    return r;
}

// g (complex [n_prob][nant]) holds the starting gains and receives the
// solution.  Dynamic LDS: two gain buffers of nant complex values.
__global__ __launch_bounds__(256) void k_cal_solve(const double *X, const double *w,
                                                    int32_t nant, double alpha, double delta,
                                                    int32_t max_iter, double *g,
                                                    int32_t *iterations, double *change) {
    extern __shared__ double lds[];
    __shared__ double red[4];
    double *ga = lds, *gb = lds + 2 * nant;
    const int64_t prob = blockIdx.x;
    const int64_t nn = (int64_t)nant * nant;
    const double *Xp = X + 2 * prob * nn;
    const double *wp = w + prob * nn;
    double *gp = g + 2 * prob * nant;
    for (int i = threadIdx.x; i < 2 * nant; i += blockDim.x) ga[i] = gp[i];
    __syncthreads();
    int it = 0;
    double last = 0.0;
    while (it < max_iter) {
        double mx = 0.0;
        for (int i = threadIdx.x; i < nant; i += blockDim.x) {
            double tr = 0.0, ti = 0.0, bot = 0.0;
            const double *Xi = Xp + 2 * (int64_t)i * nant;
            const double *wi = wp + (int64_t)i * nant;
            for (int j = 0; j < nant; ++j) {
                if (j == i) continue;
                const double gr = ga[2 * j], gi = ga[2 * j + 1];
                const double xr = Xi[2 * j], xi = Xi[2 * j + 1], ww = wi[j];
                // (g_j X_ij) w_ij
                tr += (gr * xr - gi * xi) * ww;
                ti += (gr * xi + gi * xr) * ww;
                bot += (gr * gr + gi * gi) * ww;
            }
            const double g0r = ga[2 * i], g0i = ga[2 * i + 1];
            double dr = g0r, di = g0i;
            if (bot > 0.0) {
                dr = tr / bot;
                di = ti / bot;
            }
            const double nr = (1.0 - alpha) * g0r + alpha * dr;
            const double ni = (1.0 - alpha) * g0i + alpha * di;
            gb[2 * i] = nr;
            gb[2 * i + 1] = ni;
            mx = fmax(mx, hypot(nr - g0r, ni - g0i));
        }
        last = block_max(mx, red);
        double *tmp = ga;
        ga = gb;
        gb = tmp;
        ++it;
        __syncthreads();
        if (last < delta) break;
    }
    for (int i = threadIdx.x; i < 2 * nant; i += blockDim.x) gp[i] = ga[i];
    if (threadIdx.x == 0) {
        iterations[prob] = it;
        change[prob] = last;
    }
}

hipError_t launch_cal_solve(const double *X, const double *w, int32_t nant, int64_t n_prob,
                            double alpha, double delta, int32_t max_iter, double *g,
                            int32_t *iterations, double *change, hipStream_t s) {
    if (n_prob == 0) return hipSuccess;
    const size_t lds = sizeof(double) * 4 * (size_t)nant;
    hipLaunchKernelGGL(k_cal_solve, dim3((unsigned)n_prob), dim3(256), lds, s, X, w, nant,
                       alpha, delta, max_iter, g, iterations, change);
    return hipGetLastError();
}

}  // namespace lr
