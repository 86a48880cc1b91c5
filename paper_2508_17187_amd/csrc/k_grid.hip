// The gridding / degridding hot path on gfx950 (no MFMA: the work is a
// scatter / gather, not a dense contraction).
//
// Gridding G (Eq. IMAGE-MOD) runs in two kernels over a binning plan:
//   presum   for every group of samples that share plane, kernel and
//            footprint, A_g = sum W V (exact regrouping of the sum; FP32 or
//            FP64), together with the class counters and FP64 sum of weights;
//   grid     one workgroup per chunk of the (tile, group) pairs of a 32 x 32
//            cell tile.  Each thread owns four cells of the tile and
//            accumulates Ct(o, t) phi(t) A_g over every group covering them in
//            registers; the tile is written once at the end, with plain loads
//            and stores when the chunk owns the whole tile.  Group data are
//            workgroup-uniform (scalar loads); a kernel tap is one vector load.
// Degridding D (Eq. ME-MOD-GRIDDED):
//   degrid   one wavefront per group gathers sum_t conj(Ct phi) grid over the
//            footprint (lanes over taps, coalesced along t_u) and reduces
//            across lanes;
//   expand   writes each group's value to every sample of the group (0 for
//            flagged, skipped and dropped samples).
#include <stdlib.h>

#include <algorithm>

#include "lr_internal.h"
#include "lr_launch.h"

namespace lr {

template <typename T>
struct cpx {
    T x, y;
};

__global__ void k_zero(uint4 *p, int64_t n16, uint8_t *tail, int ntail) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) p[i] = make_uint4(0, 0, 0, 0);
    if (i < ntail) tail[i] = 0;
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    int64_t n16 = (int64_t)(bytes / 16);
    int ntail = (int)(bytes - n16 * 16);
    int64_t n = n16 > ntail ? n16 : ntail;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (uint4 *)p,
                       n16, (uint8_t *)p + n16 * 16, ntail);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CF element access; f16 / bf16 pairs are decoded exactly to FP32 and
// multiplied by the plane's 2^-e.
template <int ST>
struct CFElem;
template <>
struct CFElem<LR_F64> {
    typedef double T;
    __device__ static cpx<double> load(const void *t, int64_t i, float) {
        double2 v = ((const double2 *)t)[i];
        return {v.x, v.y};
    }
};
template <>
struct CFElem<LR_F32> {
    typedef float T;
    __device__ static cpx<float> load(const void *t, int64_t i, float) {
        float2 v = ((const float2 *)t)[i];
        return {v.x, v.y};
    }
};
template <>
struct CFElem<LR_F32_CF16> {
    typedef float T;
    __device__ static cpx<float> load(const void *t, int64_t i, float sc) {
        uint32_t b = ((const uint32_t *)t)[i];
        _Float16 lo, hi;
        uint16_t l16 = (uint16_t)(b & 0xffffu), h16 = (uint16_t)(b >> 16);
        __builtin_memcpy(&lo, &l16, 2);
        __builtin_memcpy(&hi, &h16, 2);
        return {(float)lo * sc, (float)hi * sc};
    }
};
template <>
struct CFElem<LR_F32_CFBF16> {
    typedef float T;
    __device__ static cpx<float> load(const void *t, int64_t i, float sc) {
        uint32_t b = ((const uint32_t *)t)[i];
        return {__uint_as_float(b << 16) * sc, __uint_as_float(b & 0xffff0000u) * sc};
    }
};

template <typename T>
__device__ __forceinline__ void cmac(cpx<T> &acc, const cpx<T> &c, const cpx<T> &a) {
    acc.x = fma(c.x, a.x, acc.x);
    acc.x = fma(-c.y, a.y, acc.x);
    acc.y = fma(c.x, a.y, acc.y);
    acc.y = fma(c.y, a.x, acc.y);
}

// conj(c) * g accumulated
template <typename T>
__device__ __forceinline__ void cmac_conj(cpx<T> &acc, const cpx<T> &c, const cpx<T> &g) {
    acc.x = fma(c.x, g.x, acc.x);
    acc.x = fma(c.y, g.y, acc.x);
    acc.y = fma(c.x, g.y, acc.y);
    acc.y = fma(-c.y, g.x, acc.y);
}

// Pointing phasor of tap (tu, tv): f exp(-2 pi i ((tu O - ou) bu + (tv O - ov) bv)),
// argument formed and reduced modulo 1 in FP64.
template <typename T>
__device__ __forceinline__ cpx<T> phasor(const GroupMeta &gm, int tu, int tv, int O) {
    double a = fma((double)(tu * O - gm.ou), gm.bu, (double)(tv * O - gm.ov) * gm.bv);
    a = a - rint(a);
    cpx<T> r;
    if (sizeof(T) == 8) {
        double s, c;
        sincospi(-2.0 * a, &s, &c);
        r.x = (T)(gm.f * c);
        r.y = (T)(gm.f * s);
    } else {
        float s, c;
        sincospif((float)(-2.0 * a), &s, &c);
        r.x = (T)((float)gm.f * c);
        r.y = (T)((float)gm.f * s);
    }
    return r;
}

template <typename T>
__device__ __forceinline__ cpx<T> cmul(const cpx<T> &a, const cpx<T> &b) {
    cpx<T> r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

__device__ __forceinline__ float wave_sum(float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__device__ __forceinline__ long long wave_sum_ll(long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// ---------------------------------------------------------------------------
// presum + counters: one thread per sorted kept pair, a segmented scan over
// the wavefront by group, one atomic per group segment of the wave (into A,
// zeroed beforehand); threads past the kept pairs count the dropped and
// skipped ones.
template <typename T, int NPOL, bool UNIT, bool SUMS>
__global__ __launch_bounds__(256) void k_presum(
    int64_t n_kept, int64_t n_pairs, const int32_t *order, const int32_t *gidx,
    const GroupMeta *groups, const T *vis, const T *weight, cpx<T> *A, double *sumwt,
    long long *counters) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    long long kept = 0, flagged = 0, dropped = 0;
    double sw[NPOL];
    cpx<T> a[NPOL];
    for (int p = 0; p < NPOL; ++p) {
        sw[p] = 0.0;
        a[p] = {(T)0, (T)0};
    }
    int g = -1, plane = -1;
    if (i < n_kept) {
        g = gidx[i];
        plane = groups[g].plane;
        int64_t pair = order[i];
        for (int p = 0; p < NPOL; ++p) {
            T W = weight ? weight[pair * NPOL + p] : (T)1;
            if (W != (T)0) {
                ++kept;
                sw[p] = (double)W;
                if (SUMS) {
                    if (UNIT) {
                        a[p].x = W;
                    } else {
                        const T *v = vis + 2 * (pair * NPOL + p);
                        a[p].x = W * v[0];
                        a[p].y = W * v[1];
                    }
                }
            } else {
                ++flagged;
            }
        }
    } else if (i < n_pairs) {
        int32_t v = order[i];
        bool skipped = (v >> 30) & 1;
        int64_t pair = v & ~(1 << 30);
        for (int p = 0; p < NPOL; ++p) {
            T W = weight ? weight[pair * NPOL + p] : (T)1;
            if (skipped || W == (T)0) ++flagged; else ++dropped;
        }
    }
    if (SUMS) {
        // segmented inclusive scan by group id across the wavefront
        for (int off = 1; off < 64; off <<= 1) {
            int go = __shfl_up(g, off);
            bool take = lane >= off && go == g;
            for (int p = 0; p < NPOL; ++p) {
                T x = __shfl_up(a[p].x, off), y = __shfl_up(a[p].y, off);
                if (take) {
                    a[p].x += x;
                    a[p].y += y;
                }
            }
        }
        int gn = __shfl_down(g, 1);
        bool last = (lane == 63) || gn != g;
        if (g >= 0 && last)
            for (int p = 0; p < NPOL; ++p) {
                atomicAdd(&A[(int64_t)g * NPOL + p].x, a[p].x);
                if (!UNIT) atomicAdd(&A[(int64_t)g * NPOL + p].y, a[p].y);
            }
    }
    if (counters) {
        kept = wave_sum_ll(kept);
        flagged = wave_sum_ll(flagged);
        dropped = wave_sum_ll(dropped);
        if (lane == 0) {
            if (kept) atomicAdd((unsigned long long *)&counters[0], (unsigned long long)kept);
            if (flagged) atomicAdd((unsigned long long *)&counters[1], (unsigned long long)flagged);
            if (dropped) atomicAdd((unsigned long long *)&counters[2], (unsigned long long)dropped);
        }
    }
    if (sumwt) {
        // one atomic per wavefront when every lane with a sample shares its plane
        unsigned long long has = __ballot(plane >= 0);
        int lead = has ? __shfl(plane, __ffsll((long long)has) - 1) : -1;
        bool uniform = __all(plane < 0 || plane == lead);
        if (uniform) {
            for (int p = 0; p < NPOL; ++p) {
                double s = wave_sum(sw[p]);
                if (lane == 0 && lead >= 0 && s != 0.0) atomicAdd(&sumwt[lead * NPOL + p], s);
            }
        } else if (plane >= 0) {
            for (int p = 0; p < NPOL; ++p)
                if (sw[p] != 0.0) atomicAdd(&sumwt[plane * NPOL + p], sw[p]);
        }
    }
}

// ---------------------------------------------------------------------------
// The same presum walking the pairs in natural order along tracks: when the
// data repeat with a period of L pairs (time-major rows), pair c + m L is the
// next sample of the track of pair c.  A lane owns column c for TM steps and
// accumulates while its group is unchanged, flushing with atomics on a
// change; the 64 lanes of a wavefront read 64 consecutive pairs at each step.
template <typename T, int NPOL, bool UNIT, bool SUMS>
__global__ __launch_bounds__(256) void k_presum_col(
    int64_t n_pairs, int64_t L, int32_t TM, const int32_t *pair_group,
    const GroupMeta *groups, const T *vis, const T *weight, cpx<T> *A, double *sumwt,
    long long *counters) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t ncolw = (L + 63) / 64;
    const int64_t c = (wave % ncolw) * 64 + lane;
    const int64_t m0 = (wave / ncolw) * TM;
    long long kept = 0, flagged = 0, dropped = 0;
    double sw[NPOL];
    cpx<T> acc[NPOL];
    for (int p = 0; p < NPOL; ++p) {
        sw[p] = 0.0;
        acc[p] = {(T)0, (T)0};
    }
    int cur = -1, plane = -1;
    auto flush = [&]() {
        if (SUMS && cur >= 0)
            for (int p = 0; p < NPOL; ++p) {
                atomicAdd(&A[(int64_t)cur * NPOL + p].x, acc[p].x);
                if (!UNIT) atomicAdd(&A[(int64_t)cur * NPOL + p].y, acc[p].y);
            }
        for (int p = 0; p < NPOL; ++p) acc[p] = {(T)0, (T)0};
    };
    if (c < L) {
        for (int64_t m = m0; m < m0 + TM; ++m) {
            const int64_t j = c + m * L;
            if (j >= n_pairs) break;
            const int g = pair_group[j];
            if (g != cur) {
                flush();
                cur = g;
                if (g >= 0) plane = groups[g].plane;
            }
            for (int p = 0; p < NPOL; ++p) {
                T W = weight ? weight[j * NPOL + p] : (T)1;
                if (g < 0) {
                    if (g == -2 || W == (T)0) ++flagged; else ++dropped;
                } else if (W != (T)0) {
                    ++kept;
                    sw[p] += (double)W;
                    if (SUMS) {
                        if (UNIT) {
                            acc[p].x += W;
                        } else {
                            const T *v = vis + 2 * (j * NPOL + p);
                            acc[p].x = fma(W, v[0], acc[p].x);
                            acc[p].y = fma(W, v[1], acc[p].y);
                        }
                    }
                } else {
                    ++flagged;
                }
            }
        }
        flush();
    }
    if (counters) {
        kept = wave_sum_ll(kept);
        flagged = wave_sum_ll(flagged);
        dropped = wave_sum_ll(dropped);
        if (lane == 0) {
            if (kept) atomicAdd((unsigned long long *)&counters[0], (unsigned long long)kept);
            if (flagged) atomicAdd((unsigned long long *)&counters[1], (unsigned long long)flagged);
            if (dropped) atomicAdd((unsigned long long *)&counters[2], (unsigned long long)dropped);
        }
    }
    if (sumwt) {
        unsigned long long has = __ballot(plane >= 0);
        int lead = has ? __shfl(plane, __ffsll((long long)has) - 1) : -1;
        bool uniform = __all(plane < 0 || plane == lead);
        if (uniform) {
            for (int p = 0; p < NPOL; ++p) {
                double s = wave_sum(sw[p]);
                if (lane == 0 && lead >= 0 && s != 0.0) atomicAdd(&sumwt[lead * NPOL + p], s);
            }
        } else if (plane >= 0) {
            for (int p = 0; p < NPOL; ++p)
                if (sw[p] != 0.0) atomicAdd(&sumwt[plane * NPOL + p], sw[p]);
        }
    }
}

// Expand along tracks, same traversal: every pair gets its group's value
// (0 when dropped, skipped or flagged); 64 consecutive pairs per store.
template <typename T, int NPOL>
__global__ __launch_bounds__(256) void k_expand_col(int64_t n_pairs, int64_t L, int32_t TM,
                                                    const int32_t *pair_group,
                                                    const cpx<T> *Vg, cpx<T> *vis,
                                                    const T *weight) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t ncolw = (L + 63) / 64;
    const int64_t c = (wave % ncolw) * 64 + lane;
    const int64_t m0 = (wave / ncolw) * TM;
    if (c >= L) return;
    for (int64_t m = m0; m < m0 + TM; ++m) {
        const int64_t j = c + m * L;
        if (j >= n_pairs) break;
        const int g = pair_group[j];
        for (int p = 0; p < NPOL; ++p) {
            bool zero = g < 0 || (weight && weight[j * NPOL + p] == (T)0);
            vis[j * NPOL + p] = zero ? cpx<T>{(T)0, (T)0} : Vg[(int64_t)g * NPOL + p];
        }
    }
}

// Work shape of the track kernels: TM steps per lane, enough wavefronts to
// fill the chip.
static void col_shape(int64_t n_pairs, int64_t L, int32_t &TM, int64_t &blocks) {
    int64_t M = (n_pairs + L - 1) / L;
    int64_t ncolw = (L + 63) / 64;
    int64_t tm = (M * ncolw + 4095) / 4096;
    if (tm < 1) tm = 1;
    if (tm > M) tm = M;
    TM = (int32_t)tm;
    int64_t waves = ncolw * ((M + tm - 1) / tm);
    blocks = (waves + 3) / 4;
}

// ---------------------------------------------------------------------------
// Tile gridder.  One workgroup per chunk of (tile, group) pairs of one
// 32 x 32 tile; thread t owns the four cells (x0 + t % 32, y0 + t / 32 + 8 j)
// and accumulates Ct(o, t) phi(t) A_g for every group whose footprint covers
// them, in registers.  A chunk that holds all of its tile's pairs writes the
// tile with plain loads and stores; otherwise (and for the PSF's mirror
// image) the flush is atomic.
struct TileArgs {
    const GroupMeta *groups;
    const int32_t *tp_group, *chunk_start, *chunk_tile, *chunk_excl;
    const void *A;
    void *grid;
    CFView cf;
    int32_t nx, ny, ntx, nty;
    int64_t pol_stride;   // nx * ny
};

// Per-pair data of a chunk, staged in LDS once per workgroup.
struct TileItem {
    int64_t cf_off;
    int32_t bx, by;   // footprint origin p - h
    int32_t S, conj;
    float sc;         // 2^-e of the CF plane
    int32_t h;
};

// Exact t / S and t % S for 0 <= t < 2^22 through a float reciprocal.
__device__ __forceinline__ void divmod_small(int t, int S, float invS, int &q, int &r) {
    q = (int)(((float)t + 0.5f) * invS);
    r = t - q * S;
    if (r < 0) { --q; r += S; } else if (r >= S) { ++q; r -= S; }
}

template <typename T, int ST, int NPOL, bool PO, bool PSF>
__global__ __launch_bounds__(256) void k_grid_tile(TileArgs a) {
    __shared__ TileItem items[kChunkMax];
    __shared__ cpx<T> avs[kChunkMax * NPOL];
    __shared__ GroupMeta gms[PO ? kChunkMax : 1];
    const int c = blockIdx.x;
    const int32_t s0 = a.chunk_start[c];
    const int n = a.chunk_start[c + 1] - s0;
    const int32_t key = a.chunk_tile[c];
    const bool excl = !PSF && a.chunk_excl[c];
    const int tx = key % a.ntx;
    const int rest = key / a.ntx;
    const int ty = rest % a.nty;
    const int P = rest / a.nty;
    const int x = tx * kTile + (threadIdx.x & 31);
    const int yb = ty * kTile + (threadIdx.x >> 5);
    const cpx<T> *Av = (const cpx<T> *)a.A;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int32_t g = a.tp_group[s0 + t];
        const GroupMeta gm = a.groups[g];
        const int h = a.cf.h[gm.k];
        TileItem ti;
        ti.cf_off = gm.cf_off;
        ti.bx = gm.pu - h;
        ti.by = gm.pv - h;
        ti.S = 2 * h + 1;
        ti.conj = gm.conj;
        ti.sc = a.cf.scale[gm.fg * a.cf.n_w + gm.k];
        ti.h = h;
        items[t] = ti;
        for (int p = 0; p < NPOL; ++p) avs[t * NPOL + p] = Av[(int64_t)g * NPOL + p];
        if (PO) gms[t] = gm;
    }
    __syncthreads();
    cpx<T> acc[4][NPOL];
    for (int j = 0; j < 4; ++j)
        for (int p = 0; p < NPOL; ++p) acc[j][p] = {(T)0, (T)0};
    int touched = 0;
#pragma unroll 2
    for (int t = 0; t < n; ++t) {
        const TileItem ti = items[t];
        const int dx = x - ti.bx;
        const bool inx = (unsigned)dx < (unsigned)ti.S;
        cpx<T> cv[4];
        int dys[4];
        int inm = 0;
        // the four cell loads are issued together, predicated instead of branched
        for (int j = 0; j < 4; ++j) {
            const int dy = yb + 8 * j - ti.by;
            dys[j] = dy;
            const bool in = inx && (unsigned)dy < (unsigned)ti.S;
            inm |= in ? (1 << j) : 0;
            cv[j] = CFElem<ST>::load(a.cf.table, ti.cf_off + (in ? dy * ti.S + dx : 0), ti.sc);
        }
        for (int j = 0; j < 4; ++j) {
            const bool in = (inm >> j) & 1;
            if (!in) cv[j] = {(T)0, (T)0};
            if (ti.conj) cv[j].y = -cv[j].y;
            if (PO && in) cv[j] = cmul(cv[j], phasor<T>(gms[t], dx - ti.h, dys[j] - ti.h, a.cf.O));
        }
        for (int p = 0; p < NPOL; ++p) {
            const cpx<T> av = avs[t * NPOL + p];
            for (int j = 0; j < 4; ++j) cmac(acc[j][p], cv[j], av);
        }
        touched |= inm;
    }
    T *grid = (T *)a.grid;
    for (int j = 0; j < 4; ++j) {
        if (!(touched & (1 << j))) continue;
        const int y = yb + 8 * j;
        for (int p = 0; p < NPOL; ++p) {
            const int64_t base = ((int64_t)P * NPOL + p) * a.pol_stride;
            T *q = grid + 2 * (base + (int64_t)y * a.nx + x);
            if (PSF) {
                T *m = grid + 2 * (base + (int64_t)(a.ny - y) * a.nx + (a.nx - x));
                atomicAdd(q, (T)0.5 * acc[j][p].x);
                atomicAdd(q + 1, (T)0.5 * acc[j][p].y);
                atomicAdd(m, (T)0.5 * acc[j][p].x);
                atomicAdd(m + 1, -(T)0.5 * acc[j][p].y);
            } else if (excl) {
                q[0] += acc[j][p].x;
                q[1] += acc[j][p].y;
            } else {
                atomicAdd(q, acc[j][p].x);
                atomicAdd(q + 1, acc[j][p].y);
            }
        }
    }
}

// Packed variant for sparse tiles: the cells that each pair's footprint
// covers inside the tile are numbered consecutively across the chunk, thread
// t takes items t, t + 256, ..., and every item adds its npol products into an
// LDS copy of the tile with LDS atomics.  No thread idles on cells outside a
// footprint; the tile is then written once as in the register variant.
struct PackItem {
    int64_t cf_off;
    int32_t tap0;     // sub-kernel index of the first covered cell
    int32_t S, w;     // support, width of the covered rectangle
    int32_t cell0;    // tile-local index of the first covered cell
    int32_t dx0, dy0; // offsets of that cell from the footprint origin
    int32_t h, conj;
    float sc;
};

template <typename T, int ST, int NPOL, bool PO, bool PSF>
__global__ __launch_bounds__(256) void k_grid_tile_packed(TileArgs a) {
    __shared__ T accr[NPOL][kTile * kTile];
    __shared__ T acci[NPOL][kTile * kTile];
    __shared__ PackItem items[kChunkMax];
    __shared__ int32_t pre[kChunkMax + 1];
    __shared__ cpx<T> avs[kChunkMax * NPOL];
    __shared__ GroupMeta gms[PO ? kChunkMax : 1];
    const int c = blockIdx.x;
    const int32_t s0 = a.chunk_start[c];
    const int n = a.chunk_start[c + 1] - s0;
    const int32_t key = a.chunk_tile[c];
    const bool excl = !PSF && a.chunk_excl[c];
    const int tx = key % a.ntx;
    const int rest = key / a.ntx;
    const int ty = rest % a.nty;
    const int P = rest / a.nty;
    const int X0 = tx * kTile, Y0 = ty * kTile;
    const cpx<T> *Av = (const cpx<T> *)a.A;
    for (int i = threadIdx.x; i < kTile * kTile; i += blockDim.x)
        for (int p = 0; p < NPOL; ++p) {
            accr[p][i] = (T)0;
            acci[p][i] = (T)0;
        }
    int32_t cnt = 0;
    if (threadIdx.x < n) {
        const int t = threadIdx.x;
        const int32_t g = a.tp_group[s0 + t];
        const GroupMeta gm = a.groups[g];
        const int h = a.cf.h[gm.k];
        const int S = 2 * h + 1;
        const int bx = gm.pu - h, by = gm.pv - h;
        const int x0 = max(bx, X0), x1 = min(bx + S, X0 + kTile);
        const int y0 = max(by, Y0), y1 = min(by + S, Y0 + kTile);
        PackItem it;
        it.cf_off = gm.cf_off;
        it.S = S;
        it.w = x1 - x0;
        it.dx0 = x0 - bx;
        it.dy0 = y0 - by;
        it.tap0 = it.dy0 * S + it.dx0;
        it.cell0 = (y0 - Y0) * kTile + (x0 - X0);
        it.h = h;
        it.conj = gm.conj;
        it.sc = a.cf.scale[gm.fg * a.cf.n_w + gm.k];
        items[t] = it;
        cnt = (x1 - x0) * (y1 - y0);
        for (int p = 0; p < NPOL; ++p) avs[t * NPOL + p] = Av[(int64_t)g * NPOL + p];
        if (PO) gms[t] = gm;
    }
    // prefix of the covered-cell counts (n <= 64: one wavefront scan)
    if (threadIdx.x < 64) {
        int32_t v = cnt;
        for (int off = 1; off < 64; off <<= 1) {
            int32_t u = __shfl_up(v, off);
            if ((int)threadIdx.x >= off) v += u;
        }
        pre[threadIdx.x + 1] = v;
        if (threadIdx.x == 0) pre[0] = 0;
    }
    __syncthreads();
    const int32_t total = pre[n];
    int cur = 0;
    for (int32_t i = threadIdx.x; i < total; i += blockDim.x) {
        while (i >= pre[cur + 1]) ++cur;
        const PackItem it = items[cur];
        const int local = i - pre[cur];
        int cy, cx;
        divmod_small(local, it.w, 1.0f / (float)it.w, cy, cx);
        cpx<T> cv = CFElem<ST>::load(a.cf.table, it.cf_off + it.tap0 + cy * it.S + cx, it.sc);
        if (it.conj) cv.y = -cv.y;
        if (PO) cv = cmul(cv, phasor<T>(gms[cur], it.dx0 + cx - it.h, it.dy0 + cy - it.h, a.cf.O));
        const int cell = it.cell0 + cy * kTile + cx;
        for (int p = 0; p < NPOL; ++p) {
            const cpx<T> av = avs[cur * NPOL + p];
            cpx<T> r = {(T)0, (T)0};
            cmac(r, cv, av);
            atomicAdd(&accr[p][cell], r.x);
            atomicAdd(&acci[p][cell], r.y);
        }
    }
    __syncthreads();
    T *grid = (T *)a.grid;
    for (int i = threadIdx.x; i < kTile * kTile; i += blockDim.x) {
        const int x = X0 + (i & (kTile - 1)), y = Y0 + i / kTile;
        if (x >= a.nx || y >= a.ny) continue;
        for (int p = 0; p < NPOL; ++p) {
            const T vr = accr[p][i], vi = acci[p][i];
            if (vr == (T)0 && vi == (T)0) continue;
            const int64_t base = ((int64_t)P * NPOL + p) * a.pol_stride;
            T *q = grid + 2 * (base + (int64_t)y * a.nx + x);
            if (PSF) {
                T *m = grid + 2 * (base + (int64_t)(a.ny - y) * a.nx + (a.nx - x));
                atomicAdd(q, (T)0.5 * vr);
                atomicAdd(q + 1, (T)0.5 * vi);
                atomicAdd(m, (T)0.5 * vr);
                atomicAdd(m + 1, -(T)0.5 * vi);
            } else if (excl) {
                q[0] += vr;
                q[1] += vi;
            } else {
                atomicAdd(q, vr);
                atomicAdd(q + 1, vi);
            }
        }
    }
}

// ---------------------------------------------------------------------------
struct DegridArgs {
    const GroupMeta *groups;
    int64_t n_groups;
    const void *grid;
    void *Vg;
    CFView cf;
    int32_t nx, ny;
    int64_t pol_stride;
};

template <typename T, int ST, int NPOL, bool PO>
__global__ __launch_bounds__(256) void k_degrid(DegridArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (g >= a.n_groups) return;
    const GroupMeta gm = a.groups[g];
    const int h = a.cf.h[gm.k];
    const int S = 2 * h + 1;
    const int SS = S * S;
    const float invS = 1.0f / (float)S;
    const float sc = a.cf.scale[gm.fg * a.cf.n_w + gm.k];
    const T *grid = (const T *)a.grid;
    const int64_t base = gm.cell - (int64_t)h * a.nx - h;     // cell of tap (0, 0), pol 0
    cpx<T> sum[NPOL];
    for (int p = 0; p < NPOL; ++p) sum[p] = {(T)0, (T)0};
    // four taps per lane per step, their loads issued together
    for (int t0 = 0; t0 < SS; t0 += 256) {
        cpx<T> cv[4], gv[4][NPOL];
        int tys[4], txs[4];
        for (int u = 0; u < 4; ++u) {
            const int tap = t0 + u * 64 + lane;
            const bool in = tap < SS;
            int ty, tx;
            divmod_small(in ? tap : 0, S, invS, ty, tx);
            tys[u] = ty;
            txs[u] = tx;
            cv[u] = CFElem<ST>::load(a.cf.table, gm.cf_off + (in ? tap : 0), sc);
            if (!in) cv[u] = {(T)0, (T)0};
            const int64_t cell = base + (int64_t)ty * a.nx + tx;
            for (int p = 0; p < NPOL; ++p) {
                const T *q = grid + 2 * (cell + p * a.pol_stride);
                gv[u][p] = {q[0], q[1]};
            }
        }
        for (int u = 0; u < 4; ++u) {
            if (gm.conj) cv[u].y = -cv[u].y;
            if (PO && t0 + u * 64 + lane < SS)
                cv[u] = cmul(cv[u], phasor<T>(gm, txs[u] - h, tys[u] - h, a.cf.O));
            for (int p = 0; p < NPOL; ++p) cmac_conj(sum[p], cv[u], gv[u][p]);
        }
    }
    cpx<T> *out = (cpx<T> *)a.Vg;
    for (int p = 0; p < NPOL; ++p) {
        T x = wave_sum(sum[p].x), y = wave_sum(sum[p].y);
        if (lane == 0) out[g * NPOL + p] = {x, y};
    }
}

template <typename T, int NPOL>
__global__ __launch_bounds__(256) void k_expand(int64_t n_kept, int64_t n_pairs,
                                                const int32_t *order, const int32_t *gidx,
                                                const cpx<T> *Vg, cpx<T> *vis,
                                                const T *weight) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pairs) return;
    int64_t pair = order[i] & ~(1 << 30);
    if (i < n_kept) {
        int64_t g = gidx[i];
        for (int p = 0; p < NPOL; ++p) {
            bool flag = weight && weight[pair * NPOL + p] == (T)0;
            vis[pair * NPOL + p] = flag ? cpx<T>{(T)0, (T)0} : Vg[g * NPOL + p];
        }
    } else {
        for (int p = 0; p < NPOL; ++p) vis[pair * NPOL + p] = {(T)0, (T)0};
    }
}

// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <typename T, int NPOL>
static hipError_t presum_t(const lr_plan *P, const VisArgs &v, void *A, double *sumwt,
                           int64_t *counters, bool sums, hipStream_t s) {
    dim3 grd(nblk(P->n_pairs, 256)), blk(256);
    const T *vis = (const T *)v.vis;
    const T *wt = (const T *)v.weight;
    long long *cnt = (long long *)counters;
    if (sums) {
        hipError_t e = launch_zero(A, (size_t)std::max<int64_t>(P->n_groups, 1) * NPOL *
                                          sizeof(cpx<T>), s);
        if (e != hipSuccess) return e;
    }
    if (P->period > 0) {
        int32_t TM;
        int64_t nb;
        col_shape(P->n_pairs, P->period, TM, nb);
        dim3 g2((unsigned)nb);
        if (!sums)
            hipLaunchKernelGGL((k_presum_col<T, NPOL, false, false>), g2, blk, 0, s,
                               P->n_pairs, P->period, TM, P->pair_group, P->groups, vis, wt,
                               (cpx<T> *)A, sumwt, cnt);
        else if (v.unit_vis)
            hipLaunchKernelGGL((k_presum_col<T, NPOL, true, true>), g2, blk, 0, s, P->n_pairs,
                               P->period, TM, P->pair_group, P->groups, vis, wt, (cpx<T> *)A,
                               sumwt, cnt);
        else
            hipLaunchKernelGGL((k_presum_col<T, NPOL, false, true>), g2, blk, 0, s,
                               P->n_pairs, P->period, TM, P->pair_group, P->groups, vis, wt,
                               (cpx<T> *)A, sumwt, cnt);
        return hipGetLastError();
    }
    if (!sums)
        hipLaunchKernelGGL((k_presum<T, NPOL, false, false>), grd, blk, 0, s, P->n_kept,
                           P->n_pairs, P->order, P->gidx, P->groups, vis, wt, (cpx<T> *)A,
                           sumwt, cnt);
    else if (v.unit_vis)
        hipLaunchKernelGGL((k_presum<T, NPOL, true, true>), grd, blk, 0, s, P->n_kept,
                           P->n_pairs, P->order, P->gidx, P->groups, vis, wt, (cpx<T> *)A,
                           sumwt, cnt);
    else
        hipLaunchKernelGGL((k_presum<T, NPOL, false, true>), grd, blk, 0, s, P->n_kept,
                           P->n_pairs, P->order, P->gidx, P->groups, vis, wt, (cpx<T> *)A,
                           sumwt, cnt);
    return hipGetLastError();
}

template <typename T>
static hipError_t presum_np(const lr_plan *P, const VisArgs &v, void *A, double *sumwt,
                            int64_t *counters, bool sums, hipStream_t s) {
    switch (v.npol) {
        case 1: return presum_t<T, 1>(P, v, A, sumwt, counters, sums, s);
        case 2: return presum_t<T, 2>(P, v, A, sumwt, counters, sums, s);
        default: return presum_t<T, 4>(P, v, A, sumwt, counters, sums, s);
    }
}

hipError_t launch_presum(const lr_plan *P, const VisArgs &v, int precision, void *A,
                         double *sumwt, int64_t *counters, int32_t, hipStream_t s) {
    if (P->n_pairs == 0) return hipSuccess;
    if (precision == LR_F64) return presum_np<double>(P, v, A, sumwt, counters, true, s);
    return presum_np<float>(P, v, A, sumwt, counters, true, s);
}

hipError_t launch_counts(const lr_plan *P, const void *weight, int precision, int32_t npol,
                         double *sumwt, int64_t *counters, int32_t, hipStream_t s) {
    if (P->n_pairs == 0) return hipSuccess;
    VisArgs v{nullptr, weight, npol, 0};
    if (precision == LR_F64) return presum_np<double>(P, v, nullptr, sumwt, counters, false, s);
    return presum_np<float>(P, v, nullptr, sumwt, counters, false, s);
}

template <typename T, int ST, int NPOL, bool PACKED>
static hipError_t grid_t2(const TileArgs &ta, int64_t n_chunks, bool po, bool psf,
                          hipStream_t s) {
    dim3 grd((unsigned)n_chunks), blk(256);
#define LR_GRID_LAUNCH(PO_, PSF_)                                                            \
    do {                                                                                     \
        if (PACKED)                                                                          \
            hipLaunchKernelGGL((k_grid_tile_packed<T, ST, NPOL, PO_, PSF_>), grd, blk, 0, s, \
                               ta);                                                          \
        else                                                                                 \
            hipLaunchKernelGGL((k_grid_tile<T, ST, NPOL, PO_, PSF_>), grd, blk, 0, s, ta);   \
    } while (0)
    if (po) {
        if (psf) LR_GRID_LAUNCH(true, true); else LR_GRID_LAUNCH(true, false);
    } else {
        if (psf) LR_GRID_LAUNCH(false, true); else LR_GRID_LAUNCH(false, false);
    }
#undef LR_GRID_LAUNCH
    return hipGetLastError();
}

template <typename T, int ST, int NPOL>
static hipError_t grid_t(const TileArgs &ta, int64_t n_chunks, bool po, bool psf, bool packed,
                         hipStream_t s) {
    return packed ? grid_t2<T, ST, NPOL, true>(ta, n_chunks, po, psf, s)
                  : grid_t2<T, ST, NPOL, false>(ta, n_chunks, po, psf, s);
}

template <typename T, int ST>
static hipError_t grid_np(const TileArgs &ta, int64_t n_chunks, int npol, bool po, bool psf,
                          bool packed, hipStream_t s) {
    switch (npol) {
        case 1: return grid_t<T, ST, 1>(ta, n_chunks, po, psf, packed, s);
        case 2: return grid_t<T, ST, 2>(ta, n_chunks, po, psf, packed, s);
        default: return grid_t<T, ST, 4>(ta, n_chunks, po, psf, packed, s);
    }
}

// Which tile gridder: the packed one when footprints cover a small share of
// the tiles they touch, else the register one.  LR_GRIDDER=packed|register
// forces a variant (both give the same sums up to rounding order).
static bool use_packed(const lr_plan *P) {
    const char *e = getenv("LR_GRIDDER");
    if (e && e[0] == 'p') return true;
    if (e && e[0] == 'r') return false;
    double cover = (double)P->taps / ((double)P->n_tile_pairs * kTile * kTile);
    return cover < 0.5;
}

hipError_t launch_grid(const lr_plan *P, const CFView &cf, const void *A, void *grid,
                       int precision, int32_t npol, int32_t nx, int32_t ny, int32_t psf,
                       hipStream_t s) {
    if (P->n_chunks == 0) return hipSuccess;
    TileArgs ta{P->groups, P->tp_group, P->chunk_start, P->chunk_tile, P->chunk_excl, A, grid,
                cf, nx, ny, (nx + kTile - 1) / kTile, (ny + kTile - 1) / kTile,
                (int64_t)nx * ny};
    bool po = P->po != 0;
    bool pk = use_packed(P);
    int64_t nc = P->n_chunks;
    switch (precision) {
        case LR_F64: return grid_np<double, LR_F64>(ta, nc, npol, po, psf, pk, s);
        case LR_F32: return grid_np<float, LR_F32>(ta, nc, npol, po, psf, pk, s);
        case LR_F32_CF16: return grid_np<float, LR_F32_CF16>(ta, nc, npol, po, psf, pk, s);
        default: return grid_np<float, LR_F32_CFBF16>(ta, nc, npol, po, psf, pk, s);
    }
}

template <typename T, int ST, int NPOL>
static hipError_t degrid_t(const DegridArgs &da, bool po, hipStream_t s) {
    dim3 grd(nblk(da.n_groups, 4)), blk(256);
    if (po) hipLaunchKernelGGL((k_degrid<T, ST, NPOL, true>), grd, blk, 0, s, da);
    else hipLaunchKernelGGL((k_degrid<T, ST, NPOL, false>), grd, blk, 0, s, da);
    return hipGetLastError();
}

template <typename T, int ST>
static hipError_t degrid_np(const DegridArgs &da, int npol, bool po, hipStream_t s) {
    switch (npol) {
        case 1: return degrid_t<T, ST, 1>(da, po, s);
        case 2: return degrid_t<T, ST, 2>(da, po, s);
        default: return degrid_t<T, ST, 4>(da, po, s);
    }
}

hipError_t launch_degrid(const lr_plan *P, const CFView &cf, const void *grid, void *Vg,
                         int precision, int32_t npol, int32_t nx, int32_t ny, hipStream_t s) {
    if (P->n_groups == 0) return hipSuccess;
    DegridArgs da{P->groups, P->n_groups, grid, Vg, cf, nx, ny, (int64_t)nx * ny};
    bool po = P->po != 0;
    switch (precision) {
        case LR_F64: return degrid_np<double, LR_F64>(da, npol, po, s);
        case LR_F32: return degrid_np<float, LR_F32>(da, npol, po, s);
        case LR_F32_CF16: return degrid_np<float, LR_F32_CF16>(da, npol, po, s);
        default: return degrid_np<float, LR_F32_CFBF16>(da, npol, po, s);
    }
}

template <typename T>
static hipError_t expand_t(const lr_plan *P, const void *Vg, void *vis, const void *weight,
                           int npol, hipStream_t s) {
    dim3 grd(nblk(P->n_pairs, 256)), blk(256);
    const cpx<T> *V = (const cpx<T> *)Vg;
    cpx<T> *out = (cpx<T> *)vis;
    const T *w = (const T *)weight;
    if (P->period > 0) {
        int32_t TM;
        int64_t nb;
        col_shape(P->n_pairs, P->period, TM, nb);
        dim3 g2((unsigned)nb);
        const int32_t *pg = P->pair_group;
        int64_t L = P->period;
        switch (npol) {
            case 1:
                hipLaunchKernelGGL((k_expand_col<T, 1>), g2, blk, 0, s, P->n_pairs, L, TM, pg,
                                   V, out, w);
                break;
            case 2:
                hipLaunchKernelGGL((k_expand_col<T, 2>), g2, blk, 0, s, P->n_pairs, L, TM, pg,
                                   V, out, w);
                break;
            default:
                hipLaunchKernelGGL((k_expand_col<T, 4>), g2, blk, 0, s, P->n_pairs, L, TM, pg,
                                   V, out, w);
        }
        return hipGetLastError();
    }
    switch (npol) {
        case 1:
            hipLaunchKernelGGL((k_expand<T, 1>), grd, blk, 0, s, P->n_kept, P->n_pairs,
                               P->order, P->gidx, V, out, w);
            break;
        case 2:
            hipLaunchKernelGGL((k_expand<T, 2>), grd, blk, 0, s, P->n_kept, P->n_pairs,
                               P->order, P->gidx, V, out, w);
            break;
        default:
            hipLaunchKernelGGL((k_expand<T, 4>), grd, blk, 0, s, P->n_kept, P->n_pairs,
                               P->order, P->gidx, V, out, w);
    }
    return hipGetLastError();
}

hipError_t launch_expand(const lr_plan *P, const void *Vg, void *vis, const void *weight,
                         int precision, int32_t npol, hipStream_t s) {
    if (P->n_pairs == 0) return hipSuccess;
    if (precision == LR_F64) return expand_t<double>(P, Vg, vis, weight, npol, s);
    return expand_t<float>(P, Vg, vis, weight, npol, s);
}

}  // namespace lr
