// Degridding D (Eq. ME-MOD-GRIDDED): one wavefront (or a quarter of one for
// supports up to 15) per group gathers sum_t conj(Ct phi) grid over the
// footprint and reduces across lanes.
#include "k_common.h"

namespace lr {

// ---------------------------------------------------------------------------
struct DegridArgs {
    const GroupMeta *groups;
    int64_t n_groups;
    const void *grid;
    void *Vg;
    CFView cf;
    int32_t nx, ny;
    int64_t pol_stride;
    uint32_t mix;     // Mueller pass: bit q * NPOL + p adds grid pol p's gather into q (0: none)
    int32_t accum;    // add to Vg (later Mueller passes) instead of writing it
};

// A group's NPOL gathers written to Vg: as they are, or (a Mueller pass)
// correlation q gets the sum of the pols p its mask bits select, added to
// what earlier passes left when accum is set.
template <typename T, int NPOL>
__device__ __forceinline__ void store_group(const DegridArgs &a, int64_t g, const cpx<T> (&v)[NPOL]) {
    cpx<T> *out = (cpx<T> *)a.Vg + g * NPOL;
    for (int q = 0; q < NPOL; ++q) {
        cpx<T> r;
        if (a.mix == 0) {
            r = v[q];
        } else {
            r = {(T)0, (T)0};
            for (int p = 0; p < NPOL; ++p)
                if ((a.mix >> (q * NPOL + p)) & 1u) {
                    r.x += v[p].x;
                    r.y += v[p].y;
                }
        }
        if (a.accum) {
            r.x += out[q].x;
            r.y += out[q].y;
        }
        out[q] = r;
    }
}

// Taps per lane whose loads are in flight together in the degridder: 4, or
// 8 with 4-byte (FP16 / BF16) kernel values, whose raw words take half the
// registers.
constexpr int kDegridTaps = 4;

// One wavefront per group: lanes walk the footprint taps in row-major order,
// four or eight taps per lane in flight; the sub-kernel and the footprint's
// corner cell (per pol) are scalar base addresses and a lane carries 32-bit
// offsets, advanced by 64 taps at a time without division.
template <typename T, int ST, int NPOL, bool PO, bool RE>
__global__ __launch_bounds__(256) void k_degrid(DegridArgs a) {
    constexpr int E = CFRaw<ST>::bytes;
    constexpr int NT = E <= 4 ? 2 * kDegridTaps : kDegridTaps;
    typedef typename std::conditional<RE, typename CFReal<ST>::R, typename CFRaw<ST>::R>::type Raw;
    const int lane = threadIdx.x & 63;
    // consecutive groups (same plane, neighbouring footprints) run side by
    // side across the XCDs, which share the last-level cache
    const int64_t g = (int64_t)blockIdx.x * (blockDim.x >> 6) + uni(threadIdx.x >> 6);
    if (g >= a.n_groups) return;
    const GroupMeta gm = a.groups[g];
    const int h = uni(gm.h);
    const int S = 2 * h + 1;
    const int SS = S * S;
    const float sc = a.cf.scale[(int64_t)gm.fg * a.cf.n_w + gm.k];
    const bool cj = uni(gm.conj) != 0;
    const char *cfb = (const char *)a.cf.table + uni64(gm.cf_off) * E;
    // corner cell (tap (0, 0)) of pol 0
    const int64_t corner = uni64(gm.cell) - (int64_t)h * a.nx - h;
    const int64_t pstride = a.pol_stride * (int64_t)(2 * sizeof(T));
    // one scalar base per pol (its byte offset made opaque, so that a lane's
    // offset is added to it rather than folded into 64-bit vector arithmetic)
    const char *gbp[NPOL];
    for (int p = 0; p < NPOL; ++p)
        gbp[p] = (const char *)a.grid + uni64(corner * (int64_t)(2 * sizeof(T)) + p * pstride);
    const int row = a.nx * (int)(2 * sizeof(T));          // bytes per grid row
    // lane's first tap and the per-step advance of 64 taps
    const int dty = 64 / S, dtx = 64 - dty * S;
    int ty = lane / S, tx = lane - (lane / S) * S;
    int goff = ty * row + tx * (int)(2 * sizeof(T));
    cpx<T> sum[NPOL];
    for (int p = 0; p < NPOL; ++p) sum[p] = {(T)0, (T)0};
    for (int t0 = 0; t0 < SS; t0 += 64 * NT) {
        Raw cr[NT];
        cpx<T> gv[NT][NPOL];
        bool ok[NT];
        int txs[NT], tys[NT];
        for (int u = 0; u < NT; ++u) {
            const int tap = t0 + u * 64 + lane;
            ok[u] = tap < SS;
            txs[u] = tx;
            tys[u] = ty;
            // every lane loads (a lane past the footprint reads tap 0, in
            // bounds, and adds nothing): loads outside divergent branches
            // let the waits count down tap by tap
            const uint32_t co = ok[u] ? (uint32_t)tap * (uint32_t)E : 0u;
            const uint32_t go = ok[u] ? (uint32_t)goff : 0u;
            cr[u] = *(const Raw *)(cfb + co);
            for (int p = 0; p < NPOL; ++p) {
                const T *q = (const T *)(gbp[p] + go);
                gv[u][p] = {q[0], q[1]};
            }
            // advance by 64 taps
            tx += dtx;
            ty += dty;
            goff += dty * row + dtx * (int)(2 * sizeof(T));
            if (tx >= S) {
                tx -= S;
                ++ty;
                goff += row - S * (int)(2 * sizeof(T));
            }
        }
        for (int u = 0; u < NT; ++u) {
            if constexpr (RE) {
                const T c = ok[u] ? CFReal<ST>::decode(cr[u], sc) : (T)0;
                for (int p = 0; p < NPOL; ++p) {
                    sum[p].x = fma(c, gv[u][p].x, sum[p].x);
                    sum[p].y = fma(c, gv[u][p].y, sum[p].y);
                }
            } else {
                cpx<T> cv = CFRaw<ST>::decode(cr[u], sc);
                if (!ok[u]) cv = {(T)0, (T)0};
                if (cj) cv.y = -cv.y;
                if (PO) cv = cmul(cv, phasor<T>(gm, txs[u] - h, tys[u] - h, a.cf.O));
                for (int p = 0; p < NPOL; ++p) cmac_conj(sum[p], cv, gv[u][p]);
            }
        }
    }
    cpx<T> tot[NPOL];
    for (int p = 0; p < NPOL; ++p) tot[p] = {wave_sum(sum[p].x), wave_sum(sum[p].y)};
    if (lane == 0) store_group<T, NPOL>(a, g, tot);
}

// FP32 grids without a pointing phasor: lanes over pairs of neighbouring
// taps of a footprint row, so that one 16-byte load brings two grid values
// of a pol and one 16-byte (8-byte with FP16 / BF16 values) load two kernel
// values: half the vector-memory instructions of one tap per load, whose
// address processing bounds the one-tap kernel.  Pairs start at even grid
// columns (the row's first pair may begin one column before the
// footprint); with nx even a pair never crosses a grid row.  A pair's tap
// outside the footprint row reads its neighbour in the table (the row
// before or after, or the blob's padding past the table's end) and adds
// zero.
constexpr int kDegridPairs = 3;      // pairs per lane in flight

template <int ST, int NPOL, bool RE>
__global__ __launch_bounds__(256) void k_degrid_pair(DegridArgs a) {
    constexpr int E = CFRaw<ST>::bytes;                 // 8: f32, 4: f16 / bf16 pair
    typedef typename std::conditional<E == 8, f32x4_a8, u32x2_a4>::type Raw2;
    typedef typename CFRaw<ST>::R Raw;
    constexpr int NT = kDegridPairs;
    const int lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * (blockDim.x >> 6) + uni(threadIdx.x >> 6);
    if (g >= a.n_groups) return;
    const GroupMeta gm = a.groups[g];
    const int h = uni(gm.h);
    const int S = 2 * h + 1;
    const float sc = a.cf.scale[(int64_t)gm.fg * a.cf.n_w + gm.k];
    const bool cj = uni(gm.conj) != 0;
    const int lead = (uni(gm.pu) - h) & 1;              // footprint starts at an odd column
    const int W2 = (S + lead + 1) >> 1;                 // pairs per footprint row
    const int NP = S * W2;
    // kernel bytes from tap (0, -lead); grid cell (0, -lead) of pol 0
    const char *cfb = (const char *)a.cf.table + (uni64(gm.cf_off) - lead) * E;
    const int64_t corner = uni64(gm.cell) - (int64_t)h * a.nx - h - lead;
    const int64_t pstride = a.pol_stride * 8;
    const char *gbp[NPOL];
    for (int p = 0; p < NPOL; ++p)
        gbp[p] = (const char *)a.grid + uni64(corner * 8 + p * pstride);
    const int row = a.nx * 8;
    const int dr = 64 / W2, dc = 64 - dr * W2;
    int r = lane / W2, c = lane - (lane / W2) * W2;
    cpx<float> sum[NPOL];
    for (int p = 0; p < NPOL; ++p) sum[p] = {0.f, 0.f};
    for (int t0 = 0; t0 < NP; t0 += 64 * NT) {
        Raw2 cr[NT];
        f32x4_a8 gv[NT][NPOL];
        bool ok[NT], v0[NT], v1[NT];
        for (int u = 0; u < NT; ++u) {
            const int pp = t0 + u * 64 + lane;
            ok[u] = pp < NP;
            const int tu0 = 2 * c - lead;
            v0[u] = ok[u] && tu0 >= 0;
            v1[u] = ok[u] && tu0 + 1 < S;
            // lanes past the footprint load pair 0 (in bounds) and add nothing
            const uint32_t co = ok[u] ? (uint32_t)(r * S + 2 * c) * (uint32_t)E : 0u;
            const uint32_t go = ok[u] ? (uint32_t)(r * row + c * 16) : 0u;
            cr[u] = *(const Raw2 *)(cfb + co);
            for (int p = 0; p < NPOL; ++p) gv[u][p] = *(const f32x4_a8 *)(gbp[p] + go);
            c += dc;
            r += dr;
            if (c >= W2) {
                c -= W2;
                ++r;
            }
        }
        for (int u = 0; u < NT; ++u) {
            // the pair's two kernel values, zero outside the footprint row
            cpx<float> k0, k1;
            if constexpr (E == 8) {
                k0 = {cr[u].x, cr[u].y};
                k1 = {cr[u].z, cr[u].w};
            } else {
                k0 = CFRaw<ST>::decode((Raw)cr[u].x, sc);
                k1 = CFRaw<ST>::decode((Raw)cr[u].y, sc);
            }
            if (RE) k0.y = k1.y = 0.f;
            if (!v0[u]) k0 = {0.f, 0.f};
            if (!v1[u]) k1 = {0.f, 0.f};
            if (cj) {
                k0.y = -k0.y;
                k1.y = -k1.y;
            }
            for (int p = 0; p < NPOL; ++p) {
                const cpx<float> g0 = {gv[u][p].x, gv[u][p].y}, g1 = {gv[u][p].z, gv[u][p].w};
                if constexpr (RE) {
                    sum[p].x = fmaf(k0.x, g0.x, sum[p].x);
                    sum[p].y = fmaf(k0.x, g0.y, sum[p].y);
                    sum[p].x = fmaf(k1.x, g1.x, sum[p].x);
                    sum[p].y = fmaf(k1.x, g1.y, sum[p].y);
                } else {
                    cmac_conj(sum[p], k0, g0);
                    cmac_conj(sum[p], k1, g1);
                }
            }
        }
    }
    cpx<float> tot[NPOL];
    for (int p = 0; p < NPOL; ++p) tot[p] = {wave_sum(sum[p].x), wave_sum(sum[p].y)};
    if (lane == 0) store_group<float, NPOL>(a, g, tot);
}

// Small supports (S <= 2 kDegridSmallH + 1): a 7 x 7 footprint would leave
// most of a wavefront idle, so 16 lanes take one group (four groups per
// wavefront), four taps per lane in flight, and reduce over their 16 lanes.
constexpr int kDegridSmallH = 7;

template <typename T, int ST, int NPOL, bool PO, bool RE>
__global__ __launch_bounds__(256) void k_degrid_small(DegridArgs a) {
    constexpr int E = CFRaw<ST>::bytes;
    typedef typename std::conditional<RE, typename CFReal<ST>::R, typename CFRaw<ST>::R>::type Raw;
    const int sub = threadIdx.x & 15;
    const int64_t g = (int64_t)blockIdx.x * (blockDim.x >> 4) + (threadIdx.x >> 4);
    const bool live = g < a.n_groups;
    cpx<T> sum[NPOL];
    for (int p = 0; p < NPOL; ++p) sum[p] = {(T)0, (T)0};
    if (live) {
        const GroupMeta gm = a.groups[g];
        const int h = gm.h;
        const int S = 2 * h + 1;
        const int SS = S * S;
        const float invS = 1.0f / (float)S;
        const float sc = a.cf.scale[(int64_t)gm.fg * a.cf.n_w + gm.k];
        const char *cfb = (const char *)a.cf.table + gm.cf_off * E;
        const int64_t corner = gm.cell - (int64_t)h * a.nx - h;
        const T *grid = (const T *)a.grid;
        for (int t0 = 0; t0 < SS; t0 += 64) {
            Raw cr[4];
            cpx<T> gv[4][NPOL];
            int tys[4], txs[4];
            for (int u = 0; u < 4; ++u) {
                const int tap = t0 + u * 16 + sub;
                int ty, tx;
                divmod_small(tap, S, invS, ty, tx);
                tys[u] = ty;
                txs[u] = tx;
                // every lane loads (past the footprint: tap 0, in bounds,
                // adding nothing), outside divergent branches
                const bool in = tap < SS;
                const int64_t cell = in ? corner + (int64_t)ty * a.nx + tx : corner;
                cr[u] = *(const Raw *)(cfb + (in ? (int64_t)tap * E : 0));
                for (int p = 0; p < NPOL; ++p) {
                    const T *q = grid + 2 * (cell + p * a.pol_stride);
                    gv[u][p] = {q[0], q[1]};
                }
            }
            for (int u = 0; u < 4; ++u) {
                const bool in = t0 + u * 16 + sub < SS;
                if constexpr (RE) {
                    const T c = in ? CFReal<ST>::decode(cr[u], sc) : (T)0;
                    for (int p = 0; p < NPOL; ++p) {
                        sum[p].x = fma(c, gv[u][p].x, sum[p].x);
                        sum[p].y = fma(c, gv[u][p].y, sum[p].y);
                    }
                } else {
                    cpx<T> cv = CFRaw<ST>::decode(cr[u], sc);
                    if (!in) cv = {(T)0, (T)0};
                    if (gm.conj) cv.y = -cv.y;
                    if (PO) cv = cmul(cv, phasor<T>(gm, txs[u] - h, tys[u] - h, a.cf.O));
                    for (int p = 0; p < NPOL; ++p) cmac_conj(sum[p], cv, gv[u][p]);
                }
            }
        }
    }
    for (int p = 0; p < NPOL; ++p)
        for (int off = 8; off > 0; off >>= 1) {
            sum[p].x += __shfl_xor(sum[p].x, off);
            sum[p].y += __shfl_xor(sum[p].y, off);
        }
    if (live && sub == 0) store_group<T, NPOL>(a, g, sum);
}

template <typename T, int ST, int NPOL>
static hipError_t degrid_t(const DegridArgs &da, bool po, bool small, hipStream_t s) {
    dim3 blk(256);
    const bool re = !po && da.cf.real;
    if (small) {
        dim3 grd(nblk(da.n_groups, 16));
        if (po) hipLaunchKernelGGL((k_degrid_small<T, ST, NPOL, true, false>), grd, blk, 0, s, da);
        else if (re) hipLaunchKernelGGL((k_degrid_small<T, ST, NPOL, false, true>), grd, blk, 0, s, da);
        else hipLaunchKernelGGL((k_degrid_small<T, ST, NPOL, false, false>), grd, blk, 0, s, da);
        return hipGetLastError();
    }
    dim3 grd(nblk(da.n_groups, 4));
    if constexpr (sizeof(T) == 4) {
        if (!po) {
            if (re) hipLaunchKernelGGL((k_degrid_pair<ST, NPOL, true>), grd, blk, 0, s, da);
            else hipLaunchKernelGGL((k_degrid_pair<ST, NPOL, false>), grd, blk, 0, s, da);
            return hipGetLastError();
        }
    }
    if (po) hipLaunchKernelGGL((k_degrid<T, ST, NPOL, true, false>), grd, blk, 0, s, da);
    else if (re) hipLaunchKernelGGL((k_degrid<T, ST, NPOL, false, true>), grd, blk, 0, s, da);
    else hipLaunchKernelGGL((k_degrid<T, ST, NPOL, false, false>), grd, blk, 0, s, da);
    return hipGetLastError();
}

template <typename T, int ST>
static hipError_t degrid_np(const DegridArgs &da, int npol, bool po, bool small,
                            hipStream_t s) {
    switch (npol) {
        case 1: return degrid_t<T, ST, 1>(da, po, small, s);
        case 2: return degrid_t<T, ST, 2>(da, po, small, s);
        default: return degrid_t<T, ST, 4>(da, po, small, s);
    }
}

hipError_t launch_degrid(const lr_plan *P, const CFView &cf, const void *grid, void *Vg,
                         int precision, int32_t npol, int32_t nx, int32_t ny, int32_t h_max,
                         uint32_t mix, bool accum, hipStream_t s) {
    if (P->n_groups == 0) return hipSuccess;
    DegridArgs da{P->groups, P->n_groups, grid, Vg, cf, nx, ny, (int64_t)nx * ny, mix,
                  accum ? 1 : 0};
    bool po = P->po != 0;
    bool sm = h_max <= kDegridSmallH;
    switch (precision) {
        case LR_F64: return degrid_np<double, LR_F64>(da, npol, po, sm, s);
        case LR_F32: return degrid_np<float, LR_F32>(da, npol, po, sm, s);
        case LR_F32_CF16: return degrid_np<float, LR_F32_CF16>(da, npol, po, sm, s);
        default: return degrid_np<float, LR_F32_CFBF16>(da, npol, po, sm, s);
    }
}

}  // namespace lr
