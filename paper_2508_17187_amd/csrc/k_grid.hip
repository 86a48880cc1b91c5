// Gridding G (Eq. IMAGE-MOD) on gfx950 (no MFMA: the work is a scatter /
// gather, not a dense contraction), over a binning plan:
//   presum   for every group of samples that share plane, kernel and
//            footprint, A_g = sum W V (exact regrouping of the sum; FP32 or
//            FP64), together with the class counters and FP64 sum of weights;
//   grid     one workgroup per chunk of the (tile, group) pairs of a 32 x 32
//            cell tile.  Each thread owns four cells of the tile and
//            accumulates Ct(o, t) phi(t) A_g over every group covering them in
//            registers; the tile is written once at the end, with plain loads
//            and stores when the chunk owns the whole tile.  Group data are
//            workgroup-uniform (scalar loads); a kernel tap is one vector load.
//            Separable kernels of small support take the LDS-tile gridder of
//            k_sep.hip instead.
// The degridder's second half lives here too:
//   expand   writes each group's value (k_degrid.hip) to every sample of the
//            group (0 for flagged, skipped and dropped samples).
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <type_traits>

#include "lr_internal.h"
#include "lr_launch.h"
#include "k_common.h"

namespace lr {
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
// The same presum in natural order along tracks: when the data repeat with
// a period of L pairs (time-major rows), pair c + m L is the next sample of
// the track of pair c.  A wavefront covers 8 consecutive columns c x 8
// consecutive steps m (lane = 8 * step + column), so every lane issues its
// loads at once and 8 consecutive pairs are contiguous; a 3-step segmented
// shuffle reduces along the steps, and the open run of each column is
// carried from the last step of a block to the first step of the next.
// A finished run is added to A with an atomic, or simply stored when it is
// a whole group: a one-member group (kSingleton), or a single-run group
// (kSingleRun) whose run neither began before this wavefront's first step
// nor continues past its last one.  Only the groups with more than one
// member therefore need a cleared start.
// DET (deterministic order) stores those groups and sets done[g], and adds
// nothing with atomics: the other groups are summed again afterwards, in a
// fixed order, by k_presum_seg and k_presum_join.
constexpr int kColW = 8, kColT = 8, kColBlocks = 16;

template <typename T, int NPOL, bool UNIT, bool SUMS, bool DET>
__global__ __launch_bounds__(256) void k_presum_col(
    int64_t n_pairs, int64_t L, int64_t ncb, const int32_t *pair_group,
    const GroupMeta *groups, const T *vis, const T *weight, cpx<T> *A, double *sumwt,
    long long *counters, uint8_t *done) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int cl = lane & (kColW - 1), tl = lane / kColW;
    const int64_t c = (wave % ncb) * kColW + cl;
    const int64_t mw = (wave / ncb) * (kColT * kColBlocks);
    // lanes of my column, and of my column before me, in a ballot
    const uint64_t colmask = 0x0101010101010101ull << cl;
    const uint64_t below = colmask & ((1ull << lane) - 1);
    long long kept = 0, flagged = 0, dropped = 0;
    double sw[NPOL];
    cpx<T> carry[NPOL];
    for (int p = 0; p < NPOL; ++p) {
        sw[p] = 0.0;
        carry[p] = {(T)0, (T)0};
    }
    int carry_g = -1, plane = -1;
    bool carry_single = false, carry_alone = false;
    // the run holding this wavefront's first step of my column may have
    // begun in the previous wavefront: it is never stored, only added
    bool open0 = false;
    auto emit = [&](int g, bool store, const cpx<T> *v) {
        if (DET) {
            if (!store) return;
            done[g] = 1;
        }
        for (int p = 0; p < NPOL; ++p) {
            if (store) {
                A[(int64_t)g * NPOL + p] = v[p];
            } else {
                atomicAdd(&A[(int64_t)g * NPOL + p].x, v[p].x);
                if (!UNIT) atomicAdd(&A[(int64_t)g * NPOL + p].y, v[p].y);
            }
        }
    };
    // one step block in registers ahead: its loads are in flight while the
    // current block is reduced
    struct Step {
        int g;
        bool valid;
        T wv[NPOL];
        cpx<T> vv[NPOL];
    };
    auto fetch = [&](int b, Step &d) {
        const int64_t m = mw + b * kColT + tl;
        const int64_t j = c + m * L;
        d.valid = c < L && j < n_pairs;
        d.g = d.valid ? pair_group[j] : -1;
        for (int p = 0; p < NPOL; ++p) {
            d.wv[p] = (T)1;
            d.vv[p] = {(T)0, (T)0};
        }
        if (d.valid) {
            if (weight) sload(weight + j * NPOL, d.wv);
            if (SUMS && !UNIT) sload((const cpx<T> *)vis + j * NPOL, d.vv);
        }
    };
    Step nxt;
    fetch(0, nxt);
    for (int b = 0; b < kColBlocks; ++b) {
        const Step cur = nxt;
        if (b + 1 < kColBlocks) fetch(b + 1, nxt);
        cpx<T> a[NPOL];
        for (int p = 0; p < NPOL; ++p) a[p] = {(T)0, (T)0};
        const bool single = cur.g >= 0 && (cur.g & kSingleRun);
        // a one-member group's run is always whole: its sum is stored
        const bool alone = cur.g >= 0 && (cur.g & kSingleton);
        const int g = cur.g >= 0 ? (cur.g & ~kGroupFlags) : cur.g;
        if (cur.valid) {
            // the channel, hence the plane, of a lane's column is fixed
            if (g >= 0 && plane < 0) plane = groups[g].plane;
            for (int p = 0; p < NPOL; ++p) {
                const T W = cur.wv[p];
                if (g < 0) {
                    if (g == -2 || W == (T)0) ++flagged; else ++dropped;
                } else if (W != (T)0) {
                    ++kept;
                    sw[p] += (double)W;
                    if (SUMS) {
                        if (UNIT) {
                            a[p].x = W;
                        } else {
                            a[p].x = W * cur.vv[p].x;
                            a[p].y = W * cur.vv[p].y;
                        }
                    }
                } else {
                    ++flagged;
                }
            }
        }
        if (!SUMS) continue;
        if (b == 0) open0 = mw > 0 && __shfl(g, cl) >= 0;
        // the first step of a column continues the run carried from the last
        // step of the previous block, or closes it
        bool carry_ended = false;
        if (tl == 0 && carry_g >= 0) {
            if (carry_g == g) {
                for (int p = 0; p < NPOL; ++p) {
                    a[p].x += carry[p].x;
                    a[p].y += carry[p].y;
                }
            } else {
                carry_ended = true;
                emit(carry_g, (carry_single && !open0) || carry_alone, carry);
            }
        }
        const bool col_carry_ended = __shfl(carry_ended, cl);
        const int key = g >= 0 ? g : -1 - lane;     // lanes without a group never merge
        for (int off = kColW; off < 64; off <<= 1) {
            const int ko = __shfl_up(key, off);
            const bool take = lane >= off && ko == key;
            for (int p = 0; p < NPOL; ++p) {
                const T x = __shfl_up(a[p].x, off), y = __shfl_up(a[p].y, off);
                if (take) {
                    a[p].x += x;
                    a[p].y += y;
                }
            }
        }
        const int kn = __shfl_down(key, kColW);
        const bool ends = g >= 0 && tl != kColT - 1 && kn != key;   // run ended in the block
        const uint64_t endmask = __ballot(ends);
        if (ends) {
            const bool first = open0 && !col_carry_ended && !(endmask & below);
            emit(g, (single && !first) || alone, a);
        }
        if (col_carry_ended || (endmask & colmask)) open0 = false;
        // hand the last step's run to the first step of the next block
        const int src = (lane & (kColW - 1)) + (kColT - 1) * kColW;
        carry_g = __shfl(g, src);
        carry_single = __shfl(single, src);
        carry_alone = __shfl(alone, src);
        for (int p = 0; p < NPOL; ++p) {
            carry[p].x = __shfl(a[p].x, src);
            carry[p].y = __shfl(a[p].y, src);
        }
    }
    // the run still open may continue in the next wavefront
    if (SUMS && tl == 0 && carry_g >= 0) emit(carry_g, carry_alone, carry);
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

// Work shape of the track presum: ncb column blocks x ceil(M / 64) step
// blocks, one wavefront each.
static void col_shape(int64_t n_pairs, int64_t L, int64_t &ncb, int64_t &blocks) {
    int64_t M = (n_pairs + L - 1) / L;
    ncb = (L + kColW - 1) / kColW;
    const int64_t span = kColT * kColBlocks;
    int64_t waves = ncb * ((M + span - 1) / span);
    blocks = (waves + 3) / 4;
}

// ---------------------------------------------------------------------------
// Tile gridder.  One workgroup per chunk of (tile, group) pairs of one
// 32 x 32 tile; thread t owns the four cells (x0 + t % 32, y0 + 4 (t / 32) + j)
// and accumulates Ct(o, t) phi(t) A_g for every group whose footprint covers
// them, in registers.  A chunk that holds all of its tile's pairs writes the
// tile with plain stores (GRID_SET: every cell; GRID_ADD: read-modify-write
// of the touched cells); otherwise (and for the PSF's mirror image) the
// flush is atomic.  Under GRID_SET the launch has one more workgroup per
// tile after the chunks, which writes zeros when the tile has no pairs, so
// the kernel writes every cell of the grid once (shared tiles are cleared
// by the call's set-up kernel before it).
struct TileArgs {
    const GroupMeta *groups;
    const int32_t *tp_group, *chunk_start, *chunk_tile, *chunk_excl, *chunk_order, *tile_state;
    const void *A;
    void *grid;
    CFView cf;
    int32_t nx, ny, ntx, nty;
    int64_t pol_stride;   // nx * ny
    int32_t n_chunks;
    int32_t set;          // GRID_SET: exclusive chunks overwrite their whole tile
    uint32_t mix;         // Mueller pass: bit q * NPOL + p adds pol q's sum into slot p (0: none)
};

// Thread t of a 256-thread workgroup clears column t % 32 of tile `tile`.
template <typename T, int NPOL>
__device__ __forceinline__ void clear_tile(int tile, int32_t ntx, int32_t nty, int32_t nx,
                                           int32_t ny, int64_t pol_stride, cpx<T> *grid) {
    const int tx = tile % ntx;
    const int rest = tile / ntx;
    const int ty = rest % nty;
    const int P = rest / nty;
    const int x = tx * kTile + (threadIdx.x & 31);
    if (x >= nx) return;
    for (int r = threadIdx.x >> 5; r < kTile; r += blockDim.x >> 5) {
        const int y = ty * kTile + r;
        if (y >= ny) break;
        for (int p = 0; p < NPOL; ++p)
            grid[((int64_t)P * NPOL + p) * pol_stride + (int64_t)y * nx + x] = {(T)0, (T)0};
    }
}

// Per-pair data of a chunk, staged in LDS once per workgroup.
struct TileItem {
    int64_t cf_off;
    int32_t bx, by;   // footprint origin p - h
    int32_t S, conj;
    float sc;         // 2^-e of the CF plane
    int32_t h;
};

// Items a wavefront takes per step: their kernel loads are in flight
// together.
constexpr int kItemBatch = 4;
// items of a chunk as ballot bits, 64 per word
constexpr int kMaskWords = (kChunkMax + 63) / 64;

template <typename T, int ST, int NPOL, bool PO, bool PSF, bool RE, bool DET>
__global__ __launch_bounds__(256) void k_grid_tile(TileArgs a) {
    constexpr int B = kItemBatch;
    constexpr int E = CFRaw<ST>::bytes;
    typedef typename std::conditional<RE, typename CFReal<ST>::R, typename CFRaw<ST>::R>::type Raw;
    __shared__ TileItem items[kChunkMax];
    __shared__ cpx<T> avs[kChunkMax * NPOL];
    __shared__ GroupMeta gms[PO ? kChunkMax : 1];
    // workgroups take the chunks in the plan's order (largest first, or tile
    // order without chunk_order); those after the chunks (GRID_SET) clear
    // the tiles without pairs
    const int c0 = a.chunk_order && (int)blockIdx.x < a.n_chunks ? a.chunk_order[blockIdx.x]
                                                                  : (int)blockIdx.x;
    if (!PSF && c0 >= a.n_chunks) {      // GRID_SET: tiles without pairs
        const int tile = c0 - a.n_chunks;
        if (a.tile_state[tile] == 0)
            clear_tile<T, NPOL>(tile, a.ntx, a.nty, a.nx, a.ny, a.pol_stride, (cpx<T> *)a.grid);
        return;
    }
    const int32_t key = a.chunk_tile[c0];
    // DET (deterministic order): the workgroup of a tile's first chunk takes
    // all of the tile's chunks in order and owns the tile; the others exit
    if (DET && c0 > 0 && a.chunk_tile[c0 - 1] == key) return;
    const bool excl = !PSF && (DET || a.chunk_excl[c0]);
    const int tx = key % a.ntx;
    const int rest = key / a.ntx;
    const int ty = rest % a.nty;
    const int P = rest / a.nty;
    // thread t owns column t % 32 of rows 4 (t / 32) .. 4 (t / 32) + 3, so a
    // wavefront owns a band of 8 rows and skips footprints that miss it
    const int lane = threadIdx.x & 63;
    const int x = tx * kTile + (threadIdx.x & 31);
    const int yb = ty * kTile + 4 * (threadIdx.x >> 5);
    const int band0 = ty * kTile + 8 * (threadIdx.x >> 6);
    const cpx<T> *Av = (const cpx<T> *)a.A;
    cpx<T> acc[4][NPOL];
    for (int j = 0; j < 4; ++j)
        for (int p = 0; p < NPOL; ++p) acc[j][p] = {(T)0, (T)0};
    const char *table = (const char *)a.cf.table;
    for (int c = c0;;) {
        const int32_t s0 = a.chunk_start[c];
        const int n = a.chunk_start[c + 1] - s0;
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            const int32_t g = a.tp_group[s0 + t];
            const GroupMeta gm = a.groups[g];
            const int h = gm.h;
            TileItem ti;
            ti.cf_off = gm.cf_off;
            ti.bx = gm.pu - h;
            ti.by = gm.pv - h;
            ti.S = 2 * h + 1;
            ti.conj = gm.conj;
            ti.sc = a.cf.scale[(int64_t)gm.fg * a.cf.n_w + gm.k];
            ti.h = h;
            items[t] = ti;
            if (a.mix == 0) {
                for (int p = 0; p < NPOL; ++p) avs[t * NPOL + p] = Av[(int64_t)g * NPOL + p];
            } else {
                // a Mueller pass: slot p takes the sum of the correlations q
                // whose element M[q][p] is the pass's kind
                cpx<T> in[NPOL];
                for (int q = 0; q < NPOL; ++q) in[q] = Av[(int64_t)g * NPOL + q];
                for (int p = 0; p < NPOL; ++p) {
                    cpx<T> v = {(T)0, (T)0};
                    for (int q = 0; q < NPOL; ++q)
                        if ((a.mix >> (q * NPOL + p)) & 1u) {
                            v.x += in[q].x;
                            v.y += in[q].y;
                        }
                    avs[t * NPOL + p] = v;
                }
            }
            if (PO) gms[t] = gm;
        }
        __syncthreads();
        // lane i tests item i against the wavefront's band: the ballot lists the
        // items this wavefront works on (wave-uniform)
        uint64_t todo[kMaskWords];
        for (int w = 0; w < kMaskWords; ++w) {
            bool hit = false;
            const int it = w * 64 + lane;
            if (it < n) {
                const TileItem ti = items[it];
                hit = ti.by < band0 + 8 && ti.by + ti.S > band0;
            }
            todo[w] = __ballot(hit);
        }
        auto pending = [&]() {
            uint64_t any = 0;
            for (int w = 0; w < kMaskWords; ++w) any |= todo[w];
            return any != 0;
        };
        auto next = [&]() {
            for (int w = 0; w < kMaskWords; ++w)
                if (todo[w]) {
                    const int i = __builtin_ctzll(todo[w]);
                    todo[w] &= todo[w] - 1;
                    return w * 64 + i;
                }
            return -1;
        };
        while (pending()) {
            int idx[B];
            for (int b = 0; b < B; ++b) idx[b] = next();
            Raw cv[B][4];
            bool ok[B][4];
            int dxs[B], rs[B];
            float scs[B];
            // the kernel loads of the whole batch are issued before any is used;
            // an item's fields are wave-uniform, so its sub-kernel base address
            // is scalar and a lane only adds its 32-bit offset; cells outside
            // the footprint neither load nor accumulate
            for (int b = 0; b < B; ++b) {
                for (int j = 0; j < 4; ++j) ok[b][j] = false;
                dxs[b] = rs[b] = 0;
                if (idx[b] < 0) continue;
                const TileItem ti = items[idx[b]];
                const int S = uni(ti.S);
                const char *base = table + uni64(ti.cf_off) * E;
                scs[b] = ti.sc;
                const int dx = x - uni(ti.bx);
                const int r = yb - uni(ti.by);
                dxs[b] = dx;
                rs[b] = r;
                const bool cin = (unsigned)dx < (unsigned)S;
                const unsigned SS = (unsigned)(S * S);
                int off = __mul24(r, S) + dx;  // element offset of the lane's first row
                for (int j = 0; j < 4; ++j, off += S) {
                    ok[b][j] = cin && (unsigned)off < SS;
                    if (ok[b][j]) cv[b][j] = *(const Raw *)(base + (uint32_t)off * (uint32_t)E);
                }
            }
            for (int b = 0; b < B; ++b) {
                if (idx[b] < 0) continue;
                const int t = idx[b];
                const bool cj = uni(items[t].conj) != 0;
                cpx<T> av[NPOL];
                for (int p = 0; p < NPOL; ++p) av[p] = avs[t * NPOL + p];
                for (int j = 0; j < 4; ++j) {
                    if (!ok[b][j]) continue;
                    if constexpr (RE) {
                        const T c = CFReal<ST>::decode(cv[b][j], scs[b]);
                        for (int p = 0; p < NPOL; ++p) {
                            acc[j][p].x = fma(c, av[p].x, acc[j][p].x);
                            acc[j][p].y = fma(c, av[p].y, acc[j][p].y);
                        }
                    } else {
                        cpx<T> cw = CFRaw<ST>::decode(cv[b][j], scs[b]);
                        if (cj) cw.y = -cw.y;
                        if (PO) {
                            const int h = items[t].h;
                            cw = cmul(cw, phasor<T>(gms[t], dxs[b] - h, rs[b] + j - h, a.cf.O));
                        }
                        for (int p = 0; p < NPOL; ++p) cmac(acc[j][p], cw, av[p]);
                    }
                }
            }
            // every load of the batch has landed (rows that no lane needed were
            // skipped): saying so lets the next batch reuse their registers
            // without a wait in front of each load
            __builtin_amdgcn_s_waitcnt(kWaitVm0);
        }
        if (!DET || ++c >= a.n_chunks || a.chunk_tile[c] != key) break;
        __syncthreads();      // every wavefront is done with this chunk's items
    }
    T *grid = (T *)a.grid;
    const bool set = excl && a.set;
    for (int j = 0; j < 4; ++j) {
        const int y = yb + j;
        if (set) {
            if (x >= a.nx || y >= a.ny) continue;
        } else {
            // cells that received nothing are left alone (adding an exact
            // zero would not change them)
            bool any = false;
            for (int p = 0; p < NPOL; ++p)
                any |= acc[j][p].x != (T)0 || acc[j][p].y != (T)0;
            if (!any) continue;
        }
        for (int p = 0; p < NPOL; ++p) {
            const int64_t base = ((int64_t)P * NPOL + p) * a.pol_stride;
            T *q = grid + 2 * (base + (int64_t)y * a.nx + x);
            if (PSF) {
                T *m = grid + 2 * (base + (int64_t)(a.ny - y) * a.nx + (a.nx - x));
                atomicAdd(q, (T)0.5 * acc[j][p].x);
                atomicAdd(q + 1, (T)0.5 * acc[j][p].y);
                atomicAdd(m, (T)0.5 * acc[j][p].x);
                atomicAdd(m + 1, -(T)0.5 * acc[j][p].y);
            } else if (set) {
                q[0] = acc[j][p].x;
                q[1] = acc[j][p].y;
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

// Set-up of a gridding call in one launch: the first n_shared workgroups
// clear the shared tiles (GRID_SET), the rest zero up to three word spans
// (group sums, sums of weights, counters), four 8-byte words per thread.
struct SetupArgs {
    uint64_t *z[3];
    int64_t zw[3];            // words per span
    const int32_t *shared;
    int32_t n_shared, ntx, nty, nx, ny;
    int64_t pol_stride;
    void *grid;
    // group sums cleared by list (instead of span 0): the groups in multi
    uint64_t *A;
    const int32_t *multi;
    int64_t n_multi;
    int32_t gwords;           // words per group sum
    int32_t multi_blocks;
};

template <typename T, int NPOL>
__global__ __launch_bounds__(256) void k_grid_setup(SetupArgs a) {
    if ((int)blockIdx.x < a.n_shared) {
        clear_tile<T, NPOL>(a.shared[blockIdx.x], a.ntx, a.nty, a.nx, a.ny, a.pol_stride,
                            (cpx<T> *)a.grid);
        return;
    }
    const int b = (int)blockIdx.x - a.n_shared;
    if (b < a.multi_blocks) {
        const int64_t i = (int64_t)b * blockDim.x + threadIdx.x;
        if (i < a.n_multi) {
            uint64_t *q = a.A + (int64_t)a.multi[i] * a.gwords;
            for (int w = 0; w < a.gwords; ++w) q[w] = 0;
        }
        return;
    }
    int64_t w = ((int64_t)(b - a.multi_blocks) * blockDim.x + threadIdx.x) * 4;
    for (int i = 0; i < 4; ++i, ++w) {
        int64_t r = w;
        for (int k = 0; k < 3; ++k) {
            if (r < a.zw[k]) {
                a.z[k][r] = 0;
                break;
            }
            r -= a.zw[k];
        }
    }
}

// Expand: one thread per pair in natural order; the group's value comes from
// the small per-group array (0 for dropped, skipped and flagged samples).
template <typename T, int NPOL>
__global__ __launch_bounds__(256) void k_expand(int64_t n_pairs, const int32_t *pair_group,
                                                const cpx<T> *Vg, cpx<T> *vis,
                                                const T *weight) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_pairs) return;
    int g = pair_group[j];
    if (g >= 0) g &= ~kGroupFlags;
    cpx<T> out[NPOL];
    T w[NPOL];
    if (weight) sload(weight + j * NPOL, w);
    if (g >= 0) vload(Vg + (int64_t)g * NPOL, out);
    for (int p = 0; p < NPOL; ++p)
        if (g < 0 || (weight && w[p] == (T)0)) out[p] = {(T)0, (T)0};
    sstore(vis + j * NPOL, out);
}

// ---------------------------------------------------------------------------
// Deterministic mode: sums whose order does not depend on scheduling.
// Group sums over the members in the plan's sorted order (each group's
// members are consecutive there), cut into fixed segments of kDetSeg
// members, one wavefront per segment.  The wavefront takes its segment 64
// members at a time, adds each run of equal group ids with a fixed
// segmented scan over the lanes and carries the last run to the next 64.
// A group the segment holds whole is stored; a group that crosses a segment
// edge leaves its piece in part[segment][slot] (slot 0: the group began in
// an earlier segment; 1: it begins here and continues), and k_presum_join
// adds the pieces in segment order.  Groups with done[g] set (stored whole
// by the column presum) are skipped.

template <typename T, int NPOL>
__global__ __launch_bounds__(256) void k_presum_seg(int64_t n_kept, const int32_t *gidx,
                                                    const int32_t *group_start,
                                                    const int32_t *order, const T *vis,
                                                    const T *weight, const uint8_t *done,
                                                    cpx<T> *A, cpx<T> *part) {
    const int lane = threadIdx.x & 63;
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t b0 = k * kDetSeg;
    if (b0 >= n_kept) return;
    const int64_t b1 = b0 + kDetSeg < n_kept ? b0 + kDetSeg : n_kept;
    auto emit = [&](int g, const cpx<T> *v) {
        const int64_t gs = group_start[g], ge = group_start[g + 1];
        cpx<T> *dst = (gs >= b0 && ge <= b1) ? A + (int64_t)g * NPOL
                                              : part + (k * 2 + (gs < b0 ? 0 : 1)) * NPOL;
        for (int p = 0; p < NPOL; ++p) dst[p] = v[p];
    };
    int carry_g = -1;
    cpx<T> carry[NPOL];
    for (int p = 0; p < NPOL; ++p) carry[p] = {(T)0, (T)0};
    for (int64_t r0 = b0; r0 < b1; r0 += 64) {
        const int64_t i = r0 + lane;
        const bool valid = i < b1;
        const int g = valid ? gidx[i] : -1;
        const bool live = valid && !(done && done[g]);
        const int key = live ? g : -1 - lane;       // skipped lanes never merge
        cpx<T> a[NPOL];
        for (int p = 0; p < NPOL; ++p) a[p] = {(T)0, (T)0};
        if (live) {
            const int64_t pair = order[i];
            for (int p = 0; p < NPOL; ++p) {
                const T W = weight ? weight[pair * NPOL + p] : (T)1;
                if (W == (T)0) continue;
                const T *v = vis + 2 * (pair * NPOL + p);
                a[p].x = W * v[0];
                a[p].y = W * v[1];
            }
        }
        // the run carried from the previous 64 members continues here, or
        // ended there
        if (lane == 0 && carry_g >= 0) {
            if (carry_g == key) {
                for (int p = 0; p < NPOL; ++p) {
                    a[p].x = carry[p].x + a[p].x;
                    a[p].y = carry[p].y + a[p].y;
                }
            } else {
                emit(carry_g, carry);
            }
        }
        for (int off = 1; off < 64; off <<= 1) {
            const int ko = __shfl_up(key, off);
            const bool take = lane >= off && ko == key;
            for (int p = 0; p < NPOL; ++p) {
                const T x = __shfl_up(a[p].x, off), y = __shfl_up(a[p].y, off);
                if (take) {
                    a[p].x = x + a[p].x;
                    a[p].y = y + a[p].y;
                }
            }
        }
        const int kn = __shfl_down(key, 1);
        if (live && lane < 63 && kn != key) emit(g, a);
        carry_g = __shfl(key, 63);
        for (int p = 0; p < NPOL; ++p) {
            carry[p].x = __shfl(a[p].x, 63);
            carry[p].y = __shfl(a[p].y, 63);
        }
    }
    if (lane == 0 && carry_g >= 0) emit(carry_g, carry);
}

// Groups that cross a segment edge: the piece of the first segment (slot
// 1), then the later segments' pieces (slot 0), in segment order.
template <typename T, int NPOL>
__global__ __launch_bounds__(256) void k_presum_join(int64_t n_groups, const int32_t *group_start,
                                                     const uint8_t *done, const cpx<T> *part,
                                                     cpx<T> *A) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_groups || (done && done[g])) return;
    const int64_t k0 = group_start[g] / kDetSeg, k1 = (group_start[g + 1] - 1) / kDetSeg;
    if (k0 == k1) return;
    cpx<T> a[NPOL];
    for (int p = 0; p < NPOL; ++p) a[p] = part[(k0 * 2 + 1) * NPOL + p];
    for (int64_t k = k0 + 1; k <= k1; ++k)
        for (int p = 0; p < NPOL; ++p) {
            const cpx<T> q = part[k * 2 * NPOL + p];
            a[p].x += q.x;
            a[p].y += q.y;
        }
    for (int p = 0; p < NPOL; ++p) A[g * NPOL + p] = a[p];
}

// Sums of weights: block (c, k) adds the kept weights of channel c over
// rows k * 256 + t + i * 256 * kDetRowBlocks, then a fixed tree over its
// threads writes part[c][k][pol]; k_sumwt_finish adds the partials of each
// plane's channels.
template <typename T, int NPOL>
__global__ __launch_bounds__(256) void k_sumwt_part(int64_t nrow, int32_t nchan,
                                                    const int32_t *pair_group, const T *weight,
                                                    double *part) {
    __shared__ double red[256][NPOL];
    const int c = blockIdx.x / kDetRowBlocks, k = blockIdx.x % kDetRowBlocks;
    double s[NPOL];
    for (int p = 0; p < NPOL; ++p) s[p] = 0.0;
    for (int64_t r = (int64_t)k * 256 + threadIdx.x; r < nrow; r += 256 * kDetRowBlocks) {
        const int64_t j = r * nchan + c;
        if (pair_group[j] < 0) continue;          // dropped or skipped
        for (int p = 0; p < NPOL; ++p) {
            const T W = weight ? weight[j * NPOL + p] : (T)1;
            if (W != (T)0) s[p] += (double)W;
        }
    }
    for (int p = 0; p < NPOL; ++p) red[threadIdx.x][p] = s[p];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int p = 0; p < NPOL; ++p) red[threadIdx.x][p] += red[threadIdx.x + off][p];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int p = 0; p < NPOL; ++p) part[((int64_t)c * kDetRowBlocks + k) * NPOL + p] = red[0][p];
}

// One workgroup per (plane, pol): its threads add strided partials of the
// plane's channels, then a fixed tree over the threads.
__global__ __launch_bounds__(256) void k_sumwt_finish(int32_t nchan, const ChanConst *cc,
                                                      const double *part, int32_t npol,
                                                      double *sumwt) {
    __shared__ double red[256];
    const int plane = blockIdx.x / npol, p = blockIdx.x % npol;
    double s = 0.0;
    const int64_t n = (int64_t)nchan * kDetRowBlocks;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const int c = (int)(i / kDetRowBlocks);
        if (cc[c].plane == plane) s += part[i * npol + p];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) sumwt[blockIdx.x] += red[0];
}

// ---------------------------------------------------------------------------

template <typename T, int NPOL>
static hipError_t presum_t(const lr_plan *P, const VisArgs &v, void *A, double *sumwt,
                           int64_t *counters, bool sums, hipStream_t s) {
    dim3 grd(nblk(P->n_pairs, 256)), blk(256);
    const T *vis = (const T *)v.vis;
    const T *wt = (const T *)v.weight;
    long long *cnt = (long long *)counters;
    if (P->period > 0) {
        int64_t ncb, nb;
        col_shape(P->n_pairs, P->period, ncb, nb);
        dim3 g2((unsigned)nb);
        if (!sums)
            hipLaunchKernelGGL((k_presum_col<T, NPOL, false, false, false>), g2, blk, 0, s,
                               P->n_pairs, P->period, ncb, P->pair_group, P->groups, vis, wt,
                               (cpx<T> *)A, sumwt, cnt, nullptr);
        else if (v.unit_vis)
            hipLaunchKernelGGL((k_presum_col<T, NPOL, true, true, false>), g2, blk, 0, s,
                               P->n_pairs, P->period, ncb, P->pair_group, P->groups, vis, wt,
                               (cpx<T> *)A, sumwt, cnt, nullptr);
        else
            hipLaunchKernelGGL((k_presum_col<T, NPOL, false, true, false>), g2, blk, 0, s,
                               P->n_pairs, P->period, ncb, P->pair_group, P->groups, vis, wt,
                               (cpx<T> *)A, sumwt, cnt, nullptr);
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

template <typename T, int ST, int NPOL>
static hipError_t grid_t(const TileArgs &ta, int64_t n_blocks, bool po, bool psf, bool det,
                         hipStream_t s) {
    dim3 grd((unsigned)n_blocks), blk(256);
    // the point-spread function's mirror image is always flushed with
    // atomics: it has no deterministic form
    if (po) {
        if (psf) hipLaunchKernelGGL((k_grid_tile<T, ST, NPOL, true, true, false, false>), grd, blk, 0, s, ta);
        else if (det) hipLaunchKernelGGL((k_grid_tile<T, ST, NPOL, true, false, false, true>), grd, blk, 0, s, ta);
        else hipLaunchKernelGGL((k_grid_tile<T, ST, NPOL, true, false, false, false>), grd, blk, 0, s, ta);
    } else if (ta.cf.real) {
        if (psf) hipLaunchKernelGGL((k_grid_tile<T, ST, NPOL, false, true, true, false>), grd, blk, 0, s, ta);
        else if (det) hipLaunchKernelGGL((k_grid_tile<T, ST, NPOL, false, false, true, true>), grd, blk, 0, s, ta);
        else hipLaunchKernelGGL((k_grid_tile<T, ST, NPOL, false, false, true, false>), grd, blk, 0, s, ta);
    } else {
        if (psf) hipLaunchKernelGGL((k_grid_tile<T, ST, NPOL, false, true, false, false>), grd, blk, 0, s, ta);
        else if (det) hipLaunchKernelGGL((k_grid_tile<T, ST, NPOL, false, false, false, true>), grd, blk, 0, s, ta);
        else hipLaunchKernelGGL((k_grid_tile<T, ST, NPOL, false, false, false, false>), grd, blk, 0, s, ta);
    }
    return hipGetLastError();
}

template <typename T, int ST>
static hipError_t grid_np(const TileArgs &ta, int64_t n_blocks, int npol, bool po, bool psf,
                          bool det, hipStream_t s) {
    switch (npol) {
        case 1: return grid_t<T, ST, 1>(ta, n_blocks, po, psf, det, s);
        case 2: return grid_t<T, ST, 2>(ta, n_blocks, po, psf, det, s);
        default: return grid_t<T, ST, 4>(ta, n_blocks, po, psf, det, s);
    }
}

hipError_t launch_grid(const lr_plan *P, const CFView &cf, const void *A, void *grid,
                       int precision, int32_t npol, int32_t nx, int32_t ny, int32_t mode,
                       bool det, uint32_t mix, hipStream_t s) {
    const bool set = mode == GRID_SET;
    if (mix == 0 && sep_gridder(P, cf, mode, det))
        return launch_grid_sep(P, cf, A, grid, precision, npol, nx, ny, set, s);
    // GRID_SET: one more workgroup per tile clears the tiles without pairs
    const int64_t nc = P->n_chunks + (set ? P->n_tiles : 0);
    if (nc == 0) return hipSuccess;
    TileArgs ta{P->groups, P->tp_group, P->chunk_start, P->chunk_tile, P->chunk_excl,
                P->chunk_order, P->tile_state, A, grid, cf, nx, ny, (nx + kTile - 1) / kTile,
                (ny + kTile - 1) / kTile, (int64_t)nx * ny, (int32_t)P->n_chunks,
                set ? 1 : 0, mix};
    bool po = P->po != 0;
    bool psf = mode == GRID_PSF;
    det = det && !psf;
    switch (precision) {
        case LR_F64: return grid_np<double, LR_F64>(ta, nc, npol, po, psf, det, s);
        case LR_F32: return grid_np<float, LR_F32>(ta, nc, npol, po, psf, det, s);
        case LR_F32_CF16: return grid_np<float, LR_F32_CF16>(ta, nc, npol, po, psf, det, s);
        default: return grid_np<float, LR_F32_CFBF16>(ta, nc, npol, po, psf, det, s);
    }
}

template <typename T, int NPOL>
static hipError_t setup_t(const SetupArgs &sa, int64_t n_blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_grid_setup<T, NPOL>), dim3((unsigned)n_blocks), dim3(256), 0, s, sa);
    return hipGetLastError();
}

hipError_t launch_grid_setup(const lr_plan *P, void *A, size_t a_bytes, double *sumwt,
                             size_t sumwt_bytes, int64_t *counters, void *grid,
                             int precision, int32_t npol, int32_t nx, int32_t ny, bool set,
                             bool sep, hipStream_t s) {
    SetupArgs sa;
    // with a row period the track presum stores the sums of one-member
    // groups, so only the other groups are cleared
    const bool by_list = A && P->period > 0;
    sa.A = (uint64_t *)A;
    sa.multi = P->multi;
    sa.n_multi = by_list ? P->n_multi : 0;
    sa.gwords = npol * (precision == LR_F64 ? 2 : 1);
    sa.multi_blocks = (int32_t)((sa.n_multi + 255) / 256);
    sa.z[0] = (uint64_t *)A;
    sa.zw[0] = A && !by_list ? (int64_t)(a_bytes / 8) : 0;
    sa.z[1] = (uint64_t *)sumwt;
    sa.zw[1] = sumwt ? (int64_t)(sumwt_bytes / 8) : 0;
    sa.z[2] = (uint64_t *)counters;
    sa.zw[2] = counters ? 3 : 0;
    sa.shared = sep ? P->sep_shared : P->shared_tiles;
    sa.n_shared = set ? (int32_t)(sep ? P->n_sep_shared : P->n_shared) : 0;
    sa.ntx = (nx + kTile - 1) / kTile;
    sa.nty = (ny + kTile - 1) / kTile;
    sa.nx = nx;
    sa.ny = ny;
    sa.pol_stride = (int64_t)nx * ny;
    sa.grid = grid;
    const int64_t words = sa.zw[0] + sa.zw[1] + sa.zw[2];
    const int64_t n_blocks = sa.n_shared + sa.multi_blocks + (words + 1023) / 1024;
    if (n_blocks == 0) return hipSuccess;
    const bool f64 = precision == LR_F64;
    switch (npol) {
        case 1: return f64 ? setup_t<double, 1>(sa, n_blocks, s) : setup_t<float, 1>(sa, n_blocks, s);
        case 2: return f64 ? setup_t<double, 2>(sa, n_blocks, s) : setup_t<float, 2>(sa, n_blocks, s);
        default: return f64 ? setup_t<double, 4>(sa, n_blocks, s) : setup_t<float, 4>(sa, n_blocks, s);
    }
}

template <typename T>
static hipError_t expand_t(const lr_plan *P, const void *Vg, void *vis, const void *weight,
                           int npol, hipStream_t s) {
    dim3 grd(nblk(P->n_pairs, 256)), blk(256);
    const cpx<T> *V = (const cpx<T> *)Vg;
    cpx<T> *out = (cpx<T> *)vis;
    const T *w = (const T *)weight;
    switch (npol) {
        case 1:
            hipLaunchKernelGGL((k_expand<T, 1>), grd, blk, 0, s, P->n_pairs, P->pair_group, V,
                               out, w);
            break;
        case 2:
            hipLaunchKernelGGL((k_expand<T, 2>), grd, blk, 0, s, P->n_pairs, P->pair_group, V,
                               out, w);
            break;
        default:
            hipLaunchKernelGGL((k_expand<T, 4>), grd, blk, 0, s, P->n_pairs, P->pair_group, V,
                               out, w);
    }
    return hipGetLastError();
}

hipError_t launch_expand(const lr_plan *P, const void *Vg, void *vis, const void *weight,
                         int precision, int32_t npol, hipStream_t s) {
    if (P->n_pairs == 0) return hipSuccess;
    if (precision == LR_F64) return expand_t<double>(P, Vg, vis, weight, npol, s);
    return expand_t<float>(P, Vg, vis, weight, npol, s);
}

__global__ void k_clear_u8(uint8_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <typename T, int NPOL>
static hipError_t presum_det_t(const lr_plan *P, const VisArgs &v, void *A, uint8_t *done,
                               void *part, int64_t *counters, hipStream_t s) {
    dim3 blk(256);
    const T *vis = (const T *)v.vis;
    const T *wt = (const T *)v.weight;
    const bool col = P->period > 0;
    if (col) {
        // the column presum stores the groups it holds whole (and counts the
        // samples: integer atomics are exact); the rest are summed below
        int64_t ncb, nb;
        col_shape(P->n_pairs, P->period, ncb, nb);
        hipLaunchKernelGGL(k_clear_u8, dim3(nblk(P->n_groups, 256)), blk, 0, s, done,
                           P->n_groups);
        hipLaunchKernelGGL((k_presum_col<T, NPOL, false, true, true>), dim3((unsigned)nb), blk,
                           0, s, P->n_pairs, P->period, ncb, P->pair_group, P->groups, vis, wt,
                           (cpx<T> *)A, (double *)nullptr, (long long *)counters, done);
    } else if (counters) {
        VisArgs w{nullptr, v.weight, v.npol, 0};
        hipError_t e = presum_np<T>(P, w, nullptr, nullptr, counters, false, s);
        if (e != hipSuccess) return e;
    }
    if (P->n_kept == 0) return hipGetLastError();
    const uint8_t *dn = col ? done : nullptr;
    const int64_t n_seg = (P->n_kept + kDetSeg - 1) / kDetSeg;
    hipLaunchKernelGGL((k_presum_seg<T, NPOL>), dim3(nblk(n_seg * 64, 256)), blk, 0, s,
                       P->n_kept, P->gidx, P->group_start, P->order, vis, wt, dn, (cpx<T> *)A,
                       (cpx<T> *)part);
    hipLaunchKernelGGL((k_presum_join<T, NPOL>), dim3(nblk(P->n_groups, 256)), blk, 0, s,
                       P->n_groups, P->group_start, dn, (const cpx<T> *)part, (cpx<T> *)A);
    return hipGetLastError();
}

hipError_t launch_presum_det(const lr_plan *P, const VisArgs &v, int precision, void *A,
                             uint8_t *done, void *part, int64_t *counters, hipStream_t s) {
    if (P->n_pairs == 0) return hipSuccess;
    const bool f64 = precision == LR_F64;
    switch (v.npol) {
        case 1: return f64 ? presum_det_t<double, 1>(P, v, A, done, part, counters, s)
                           : presum_det_t<float, 1>(P, v, A, done, part, counters, s);
        case 2: return f64 ? presum_det_t<double, 2>(P, v, A, done, part, counters, s)
                           : presum_det_t<float, 2>(P, v, A, done, part, counters, s);
        default: return f64 ? presum_det_t<double, 4>(P, v, A, done, part, counters, s)
                            : presum_det_t<float, 4>(P, v, A, done, part, counters, s);
    }
}

template <typename T, int NPOL>
static void sumwt_part_t(const lr_plan *P, const void *weight, double *part, hipStream_t s) {
    hipLaunchKernelGGL((k_sumwt_part<T, NPOL>), dim3((unsigned)(P->nchan * kDetRowBlocks)),
                       dim3(256), 0, s, P->nrow, P->nchan, P->pair_group, (const T *)weight,
                       part);
}

hipError_t launch_sumwt_det(const lr_plan *P, const void *weight, int precision, int32_t npol,
                            int32_t nplane, double *part, double *sumwt, hipStream_t s) {
    if (P->n_pairs == 0 || !sumwt) return hipSuccess;
    const bool f64 = precision == LR_F64;
    switch (npol) {
        case 1: f64 ? sumwt_part_t<double, 1>(P, weight, part, s) : sumwt_part_t<float, 1>(P, weight, part, s); break;
        case 2: f64 ? sumwt_part_t<double, 2>(P, weight, part, s) : sumwt_part_t<float, 2>(P, weight, part, s); break;
        default: f64 ? sumwt_part_t<double, 4>(P, weight, part, s) : sumwt_part_t<float, 4>(P, weight, part, s);
    }
    hipLaunchKernelGGL(k_sumwt_finish, dim3((unsigned)(nplane * npol)), dim3(256), 0, s,
                       P->nchan, P->cc, part, npol, sumwt);
    return hipGetLastError();
}

}  // namespace lr
