// Gridder for separable kernels of small support (PS-only tables), with
// band-owned wavefronts accumulating a 32 x 32 tile in LDS.
#include <stdlib.h>
#include <string.h>

#include <type_traits>

#include "k_common.h"

namespace lr {

// ---------------------------------------------------------------------------
// Gridder for separable kernels of small support (the Standard kernel: PS
// only, one plane, S = 2h + 1 <= 15).  One workgroup owns one 32 x 32 tile:
// it accumulates the tile in LDS and writes it to the grid once, so no cell
// is updated twice in global memory and no atomics reach the grid.
//
// CF cache: a separable plane is an outer product, C[o_v][o_u][t_v][t_u] =
// cv[o_v][t_v] cu[o_u][t_u] with cu the o_v = 0, t_v = 0 row and cv the
// o_u = 0, t_u = 0 column over the centre tap.  The workgroup derives both
// factor tables ((O + 1) S values each) from the stored plane into LDS, so
// no tap is read from global memory.
//
// Each wavefront owns a band of kSepBand tile rows and is the only one to
// touch them in LDS, so its adds are plain read-modify-writes (LDS float
// atomics, which every wavefront of the tile would otherwise need, cost
// four times the rest of the kernel on one-sample groups).  The plan sorts
// a tile's pairs by pixel row, so the pairs whose footprints meet a band
// are one contiguous range, found by a wavefront-wide search; a pair whose
// footprint spans two bands is gridded by both wavefronts, each keeping
// its own rows.  The wavefront takes its range in blocks of 16 (lane l
// holds pair l & 15; the loads of the next block are in flight while one
// is gridded), one pair at a time with lanes over taps: lane t adds cu cv
// A[pol] into registers for tap t (and t + 64, ... for S > 7).  Pairs of
// one pixel (same footprint) follow each other; the registers are added to
// the band when the pixel changes.
struct SepArgs {
    const int32_t *tp_group;
    const int32_t *tile_tp;
    const int4 *part;         // (tile, first pair, end pair, several parts)
    int32_t n_parts;
    const int64_t *geo;
    const void *A;
    void *grid;
    const void *table;        // element 0 of plane (0, 0)
    const float *scale;       // 2^-e of plane (0, 0)
    int32_t O, h;
    int32_t nx, ny, ntx, nty;
    int64_t pol_stride;
    int32_t set;              // GRID_SET: every cell written (0 where nothing lands)
};

constexpr int kSepBlock = 16;

template <typename T>
__device__ __forceinline__ T lane_value(T v, int j) {
    if constexpr (sizeof(T) == 4) {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
    } else {
        const int lo = __builtin_amdgcn_readlane(__double2loint(v), j);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(v), j);
        return __hiloint2double(hi, lo);
    }
}

// FP32 broadcasts: lanes 16 r + J of every row of 16 lanes hold the same
// value (the block's pair J), and the DPP row_newbcast:J operand hands it to
// every lane of the row, so a pair's values reach all lanes with no
// instruction of their own.  A DPP read needs two wait states after a VALU
// write of its source register (s_nop 1).
// acc[p] += A[p] of the block's pair J times t, for the NPOL complex values
// of one cell, in one block: a single s_nop 1 covers every DPP source (no
// instruction inside the block writes one; the accumulators are not DPP
// operands).
#define LR_FMAC_DPP(d, v) "v_fmac_f32_dpp %" #d ", %" #v ", %[t] row_newbcast:%[j] row_mask:0xf bank_mask:0xf\n\t"
template <int J, int NPOL>
__device__ __forceinline__ void fmac_bcast_cell(cpx<float> *acc, const cpx<float> *av, float t) {
    if constexpr (NPOL == 4) {
        asm("s_nop 1\n\t" LR_FMAC_DPP(0, 8) LR_FMAC_DPP(1, 9) LR_FMAC_DPP(2, 10)
            LR_FMAC_DPP(3, 11) LR_FMAC_DPP(4, 12) LR_FMAC_DPP(5, 13) LR_FMAC_DPP(6, 14)
            LR_FMAC_DPP(7, 15)
            : "+v"(acc[0].x), "+v"(acc[0].y), "+v"(acc[1].x), "+v"(acc[1].y), "+v"(acc[2].x),
              "+v"(acc[2].y), "+v"(acc[3].x), "+v"(acc[3].y)
            : "v"(av[0].x), "v"(av[0].y), "v"(av[1].x), "v"(av[1].y), "v"(av[2].x),
              "v"(av[2].y), "v"(av[3].x), "v"(av[3].y), [t] "v"(t), [j] "n"(J));
    } else if constexpr (NPOL == 2) {
        asm("s_nop 1\n\t" LR_FMAC_DPP(0, 4) LR_FMAC_DPP(1, 5) LR_FMAC_DPP(2, 6) LR_FMAC_DPP(3, 7)
            : "+v"(acc[0].x), "+v"(acc[0].y), "+v"(acc[1].x), "+v"(acc[1].y)
            : "v"(av[0].x), "v"(av[0].y), "v"(av[1].x), "v"(av[1].y), [t] "v"(t), [j] "n"(J));
    } else {
        asm("s_nop 1\n\t" LR_FMAC_DPP(0, 2) LR_FMAC_DPP(1, 3)
            : "+v"(acc[0].x), "+v"(acc[0].y)
            : "v"(av[0].x), "v"(av[0].y), [t] "v"(t), [j] "n"(J));
    }
}
#undef LR_FMAC_DPP
template <int J>
__device__ __forceinline__ float bcast(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + J, 0xF, 0xF, true));
}
template <int J>
__device__ __forceinline__ int bcast(int v) {
    return __builtin_amdgcn_mov_dpp(v, 0x150 + J, 0xF, 0xF, true);
}

// f(integral_constant<int, J>) for J = 0 .. N - 1, in order.
template <int J, int N, typename F>
__device__ __forceinline__ void for_const(F &&f) {
    f(std::integral_constant<int, J>{});
    if constexpr (J + 1 < N) for_const<J + 1, N>(f);
}

constexpr int kSepBand = 8;                       // tile rows per wavefront
constexpr int kSepThreads = 64 * (kTile / kSepBand);

// First index i in [lo, hi) whose pair's pixel row is >= key (hi if none),
// the rows ascending over the range: 64 samples per round, so a part of
// up to 4096 pairs takes two rounds.  Wave-uniform result.
__device__ __forceinline__ int band_bound(const int32_t *tp_group, const int64_t *geo, int lo,
                                          int hi, int key, int lane) {
    while (lo < hi) {
        const int step = (hi - lo + 63) / 64;
        const int i = lo + lane * step;
        bool ge = true;                                   // past the end counts as >= key
        if (i < hi) ge = (int)((geo[tp_group[i]] >> 16) & 0xFFFF) >= key;
        const uint64_t m = __ballot(ge);
        if (m == 0) {
            lo += 63 * step + 1;
            continue;
        }
        const int c = __builtin_ctzll(m);
        if (c == 0) return lo;
        hi = min(hi, lo + c * step);
        lo += (c - 1) * step + 1;
    }
    return lo;
}

template <typename T, int ST, int NPOL, int NT>
__global__ __launch_bounds__(kSepThreads) void k_grid_sep(SepArgs a) {
    constexpr int E = CFRaw<ST>::bytes;
    typedef typename CFReal<ST>::R Raw;
    constexpr int NC = 2 * NPOL;              // values per cell
    constexpr int RS = kTile * NC + 1;        // LDS row stride: rows start one bank apart
    __shared__ T tl[kTile * RS];
    extern __shared__ __align__(16) char cf_lds[];
    // workgroups take the parts (heaviest tiles first); those after the
    // parts write the tiles without pairs as zeros (GRID_SET)
    int tile, b0, b1, shared = 0;
    if ((int)blockIdx.x < a.n_parts) {
        const int4 pt = a.part[blockIdx.x];
        tile = pt.x;
        b0 = pt.y;
        b1 = pt.z;
        shared = pt.w;
    } else {
        tile = (int)blockIdx.x - a.n_parts;
        b0 = b1 = 0;
        if (a.tile_tp[tile] != a.tile_tp[tile + 1]) return;
    }
    const int tx = tile % a.ntx;
    const int rest = tile / a.ntx;
    const int ty = rest % a.nty;
    const int P = rest / a.nty;
    const int x0 = tx * kTile, y0 = ty * kTile;
    T *grid = (T *)a.grid;
    const int lane = threadIdx.x & 63;
    if (b0 == b1) {
        // no pairs: under GRID_SET the tile is written as zeros
        if (!a.set) return;
        for (int i = threadIdx.x; i < kTile * kTile * NPOL; i += blockDim.x) {
            const int p = i % NPOL, c = i / NPOL;
            const int x = x0 + c % kTile, y = y0 + c / kTile;
            if (x < a.nx && y < a.ny) {
                T *q = grid + 2 * (((int64_t)P * NPOL + p) * a.pol_stride + (int64_t)y * a.nx + x);
                q[0] = (T)0;
                q[1] = (T)0;
            }
        }
        return;
    }
    const int h = a.h, S = 2 * h + 1, O = a.O, no = O + 1, half = O >> 1;
    T *cu = (T *)cf_lds;
    T *cv = cu + no * S;
    // this wavefront's band and the pairs whose footprints meet it (the
    // search's loads overlap the factor tables' build)
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int yb = wv * kSepBand;
    const int r0 = band_bound(a.tp_group, a.geo, b0, b1, y0 + yb - h, lane);
    const int r1 = band_bound(a.tp_group, a.geo, r0, b1, y0 + yb + kSepBand + h, lane);
    {
        const char *tb = (const char *)a.table;
        const float sc = a.scale[0];
        auto ent = [&](int ovi, int oui, int tvi, int tui) {
            const int64_t e = (((int64_t)ovi * no + oui) * S + tvi) * S + tui;
            return (T)CFReal<ST>::decode(*(const Raw *)(tb + e * E), sc);
        };
        const T centre = ent(half, half, h, h);
        for (int i = threadIdx.x; i < no * S; i += blockDim.x) {
            const int o = i / S, t = i - o * S;
            cu[i] = ent(half, o, h, t);
            cv[i] = ent(o, half, t, h) / centre;
        }
        for (int i = threadIdx.x; i < kTile * RS; i += blockDim.x) tl[i] = (T)0;
    }
    __syncthreads();
    // this lane's taps t = lane + 64 n: (tv, tu) and whether t < S^2
    int tu[NT], tv[NT];
    bool tin[NT];
    for (int n = 0; n < NT; ++n) {
        const int t = lane + 64 * n;
        tv[n] = t / S;
        tu[n] = t - tv[n] * S;
        tin[n] = t < S * S;
        if (!tin[n]) tu[n] = tv[n] = 0;
    }
    const int nb = (r1 - r0 + kSepBlock - 1) / kSepBlock;
    const cpx<T> *Av = (const cpx<T> *)a.A;
    // the band cells under the current run's footprint, in registers: read
    // from LDS when the run's pixel starts, written back when it ends (the
    // lane's tap is the cell; lanes outside the band or the tile keep
    // theirs out of LDS)
    cpx<T> acc[NT][NPOL];
    bool in[NT];
    int loff[NT], addr[NT];
    for (int n = 0; n < NT; ++n) {
        loff[n] = tv[n] * RS + tu[n] * NC;
        addr[n] = 0;
        in[n] = false;
        for (int p = 0; p < NPOL; ++p) acc[n][p] = {(T)0, (T)0};
    }
    int cur = -1;            // packed pixel of the run in the registers (wave-uniform)
    auto store_run = [&]() {
        for (int n = 0; n < NT; ++n) {
            if (in[n]) {
                T *c = tl + addr[n];
                for (int p = 0; p < NPOL; ++p) {
                    c[2 * p] = acc[n][p].x;
                    c[2 * p + 1] = acc[n][p].y;
                }
            }
        }
    };
    auto load_run = [&](int pj) {
        const int px = (pj & 0xFFFF) - h - x0, py = (pj >> 16) - h - y0;
        const int base = py * RS + px * NC;
        for (int n = 0; n < NT; ++n) {
            in[n] = tin[n] && (unsigned)(px + tu[n]) < (unsigned)kTile &&
                    (unsigned)(py + tv[n] - yb) < (unsigned)kSepBand;
            addr[n] = base + loff[n];
            if (in[n]) {
                const T *c = tl + addr[n];
                for (int p = 0; p < NPOL; ++p) acc[n][p] = {c[2 * p], c[2 * p + 1]};
            }
        }
    };
    // block loads: group, geometry and group sums of pair (l & 15)
    struct Blk {
        int64_t geo;
        cpx<T> av[NPOL];
    };
    auto load_group = [&](int blk) {
        const int i = r0 + blk * kSepBlock + (lane & (kSepBlock - 1));
        return i < r1 ? a.tp_group[i] : -1;
    };
    auto load_blk = [&](int g, Blk &d) {
        if (g >= 0) {
            d.geo = a.geo[g];
            vload(Av + (int64_t)g * NPOL, d.av);
        } else {
            d.geo = 0;
            for (int p = 0; p < NPOL; ++p) d.av[p] = {(T)0, (T)0};
        }
    };
    int g_next = 1 < nb ? load_group(1) : -1;
    Blk cb;
    if (nb > 0) load_blk(load_group(0), cb);
    for (int blk = 0; blk < nb; ++blk) {
        // the next block's sums and geometry, and the group ids of the one
        // after, are loaded while this block is gridded
        Blk nbk;
        if (blk + 1 < nb) load_blk(g_next, nbk);
        const int g_after = blk + 2 < nb ? load_group(blk + 2) : -1;
        const int cnt = min(kSepBlock, r1 - (r0 + blk * kSepBlock));
        // per-pair base addresses of the factor tables
        const int ou = (int)(int16_t)(cb.geo >> 32), ov = (int)(int16_t)(cb.geo >> 48);
        const int pix = (int)(cb.geo & 0xFFFFFFFF);
        const int ub = (ou + half) * S, vb = (ov + half) * S;
        // this lane's taps of every pair of the block, all LDS reads in
        // flight before the first is used
        T tp[kSepBlock][NT], tq[kSepBlock][NT];
        for_const<0, kSepBlock>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            int ubj, vbj;
            if constexpr (sizeof(T) == 4) {
                ubj = bcast<j>(ub);
                vbj = bcast<j>(vb);
            } else {
                ubj = __builtin_amdgcn_readlane(ub, j);
                vbj = __builtin_amdgcn_readlane(vb, j);
            }
            for (int n = 0; n < NT; ++n) {
                tp[j][n] = cu[ubj + tu[n]];
                tq[j][n] = cv[vbj + tv[n]];
            }
        });
        // every factor read is issued before any is used (the compiler would
        // otherwise wait for each pair's reads in turn), then the taps
        for (int j = 0; j < kSepBlock; ++j)
            for (int n = 0; n < NT; ++n) asm volatile("" : "+v"(tp[j][n]), "+v"(tq[j][n]));
        for (int j = 0; j < kSepBlock; ++j)
            for (int n = 0; n < NT; ++n) tp[j][n] *= tq[j][n];
        for_const<0, kSepBlock>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            if (j >= cnt) return;
            const int pj = __builtin_amdgcn_readlane(pix, j);
            if (pj != __builtin_amdgcn_readfirstlane(cur)) {
                if (cur >= 0) store_run();
                load_run(pj);
                cur = pj;
            }
            for (int n = 0; n < NT; ++n) {
                const T tap = tp[j][n];
                if constexpr (sizeof(T) == 4) {
                    fmac_bcast_cell<j, NPOL>(acc[n], cb.av, tap);
                } else {
                    for (int p = 0; p < NPOL; ++p) {
                        const T ax = lane_value(cb.av[p].x, j), ay = lane_value(cb.av[p].y, j);
                        acc[n][p].x = fma(tap, ax, acc[n][p].x);
                        acc[n][p].y = fma(tap, ay, acc[n][p].y);
                    }
                }
            }
        });
        cb = nbk;
        g_next = g_after;
    }
    if (cur >= 0) store_run();
    // write the band (only this wavefront wrote it, so no barrier): lane
    // pairs (cell, pol) with pol fastest, so LDS reads are consecutive and
    // each pol's cells are 16 consecutive grid values
    constexpr int CPI = 64 / NPOL;                 // cells per wavefront step
    for (int c0 = 0; c0 < kSepBand * kTile; c0 += CPI) {
        const int c = c0 + lane / NPOL, p = lane % NPOL;
        const int xl = c % kTile, yl = yb + c / kTile;
        const int x = x0 + xl, y = y0 + yl;
        if (x >= a.nx || y >= a.ny) continue;
        const T *src = tl + yl * RS + xl * NC + 2 * p;
        const T vx = src[0], vy = src[1];
        T *q = grid + 2 * (((int64_t)P * NPOL + p) * a.pol_stride + (int64_t)y * a.nx + x);
        if (shared) {
            // a tile split into several parts: every part adds its share
            if (vx != (T)0 || vy != (T)0) {
                atomicAdd(q, vx);
                atomicAdd(q + 1, vy);
            }
        } else if (a.set) {
            q[0] = vx;
            q[1] = vy;
        } else if (vx != (T)0 || vy != (T)0) {
            q[0] += vx;
            q[1] += vy;
        }
    }
}

template <typename T, int ST, int NPOL>
static hipError_t grid_sep_t(const SepArgs &sa, int64_t n_blocks, int S, hipStream_t s) {
    dim3 grd((unsigned)n_blocks), blk(kSepThreads);
    const size_t lds = 2 * sizeof(T) * (size_t)(sa.O + 1) * S;
    const int nt = (S * S + 63) / 64;
    if (nt <= 1) hipLaunchKernelGGL((k_grid_sep<T, ST, NPOL, 1>), grd, blk, lds, s, sa);
    else if (nt == 2) hipLaunchKernelGGL((k_grid_sep<T, ST, NPOL, 2>), grd, blk, lds, s, sa);
    else if (nt == 3) hipLaunchKernelGGL((k_grid_sep<T, ST, NPOL, 3>), grd, blk, lds, s, sa);
    else hipLaunchKernelGGL((k_grid_sep<T, ST, NPOL, 4>), grd, blk, lds, s, sa);
    return hipGetLastError();
}

template <typename T, int ST>
static hipError_t grid_sep_np(const SepArgs &sa, int64_t n_blocks, int npol, int S,
                              hipStream_t s) {
    switch (npol) {
        case 1: return grid_sep_t<T, ST, 1>(sa, n_blocks, S, s);
        case 2: return grid_sep_t<T, ST, 2>(sa, n_blocks, S, s);
        default: return grid_sep_t<T, ST, 4>(sa, n_blocks, S, s);
    }
}

bool sep_gridder(const lr_plan *P, const CFView &cf, int32_t mode, bool det) {
    if (mode == GRID_PSF || det || P->po || !cf.real || cf.n_w != 1) return false;
    static const int forced = [] {
        const char *e = getenv("LR_GRIDDER");
        if (!e) return 0;
        if (!strcmp(e, "sep")) return 1;
        if (!strcmp(e, "tile")) return -1;
        return 0;
    }();
    if (forced < 0) return false;
    // a real table with one w-plane and one frequency group: a single plane,
    // and a tile's pairs sorted by pixel row alone (the sort key puts the
    // frequency group ahead of the pixel)
    return cf.n_fg == 1 && cf.h0 <= 7;
}

hipError_t launch_grid_sep(const lr_plan *P, const CFView &cf, const void *A, void *grid,
                           int precision, int32_t npol, int32_t nx, int32_t ny, bool set,
                           hipStream_t s) {
    const int64_t n_blocks = P->n_sep_parts + (set ? P->n_tiles : 0);
    if (n_blocks == 0) return hipSuccess;
    SepArgs sa{P->tp_group, P->tile_tp, P->sep_part, (int32_t)P->n_sep_parts, P->geo, A, grid,
               nullptr, cf.scale, cf.O, cf.h0, nx, ny, (nx + kTile - 1) / kTile,
               (ny + kTile - 1) / kTile, (int64_t)nx * ny, set ? 1 : 0};
    const int S = 2 * cf.h0 + 1;
    switch (precision) {
        case LR_F64:
            sa.table = (const char *)cf.table + cf.off0 * 16;
            return grid_sep_np<double, LR_F64>(sa, n_blocks, npol, S, s);
        case LR_F32:
            sa.table = (const char *)cf.table + cf.off0 * 8;
            return grid_sep_np<float, LR_F32>(sa, n_blocks, npol, S, s);
        case LR_F32_CF16:
            sa.table = (const char *)cf.table + cf.off0 * 4;
            return grid_sep_np<float, LR_F32_CF16>(sa, n_blocks, npol, S, s);
        default:
            sa.table = (const char *)cf.table + cf.off0 * 4;
            return grid_sep_np<float, LR_F32_CFBF16>(sa, n_blocks, npol, S, s);
    }
}

}  // namespace lr
