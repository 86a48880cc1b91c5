// Binning of (row, channel) pairs (the PreSolvePrep re-ordering): index map,
// 64-bit sort keys, radix sort, grouping of identical samples and the
// decomposition of the gridder's work into wavefront tasks.
#include <string.h>

#include <cstring>

#include <rocprim/rocprim.hpp>

#include "lr_internal.h"
#include "lr_launch.h"

namespace lr {

// ---------------------------------------------------------------------------
// Small host arrays reach the device through kernel arguments, so no host
// buffer has to outlive an asynchronous copy.
struct ChanUpload {
    ChanConst c[kMaxChanPerUpload];
    int32_t n, base;
};

__global__ void k_upload_chan(ChanUpload up, ChanConst *dst) {
    int i = threadIdx.x;
    if (i < up.n) dst[up.base + i] = up.c[i];
}

struct WordUpload {
    uint32_t w[512];
    int32_t n, base;
};

__global__ void k_upload_words(WordUpload up, uint32_t *dst) {
    for (int i = threadIdx.x; i < up.n; i += blockDim.x) dst[up.base + i] = up.w[i];
}

hipError_t upload_chan(const std::vector<ChanConst> &cc, ChanConst *d, hipStream_t s) {
    for (size_t b = 0; b < cc.size(); b += kMaxChanPerUpload) {
        ChanUpload up;
        up.n = (int32_t)std::min<size_t>(kMaxChanPerUpload, cc.size() - b);
        up.base = (int32_t)b;
        for (int i = 0; i < up.n; ++i) up.c[i] = cc[b + i];
        hipLaunchKernelGGL(k_upload_chan, dim3(1), dim3(64), 0, s, up, d);
    }
    return hipGetLastError();
}

hipError_t upload_words(const void *src, size_t bytes, void *d, hipStream_t s) {
    const uint32_t *w = (const uint32_t *)src;
    size_t n = bytes / 4;
    for (size_t b = 0; b < n; b += 512) {
        WordUpload up;
        up.n = (int32_t)std::min<size_t>(512, n - b);
        up.base = (int32_t)b;
        for (int i = 0; i < up.n; ++i) up.w[i] = w[b + i];
        hipLaunchKernelGGL(k_upload_words, dim3(1), dim3(256), 0, s, up, (uint32_t *)d);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The channel constants travel by value, `up.n` channels from `up.base`.
__global__ void k_debug_map(int64_t nrow, int32_t nchan, const double *uvw, ChanUpload up,
                            MapGeom g, int32_t *out) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nrow * up.n) return;
    int64_t r = j / up.n;
    int32_t cl = (int32_t)(j - r * up.n);
    int32_t c = up.base + cl;
    int64_t i = r * nchan + c;
    ChanConst ch = up.c[cl];
    Map m = map_sample(uvw[3 * r], uvw[3 * r + 1], uvw[3 * r + 2], ch, g);
    int32_t *o = out + 8 * i;
    o[0] = m.pu; o[1] = m.pv; o[2] = m.ou; o[3] = m.ov;
    o[4] = m.k; o[5] = m.conj; o[6] = m.keep; o[7] = ch.fg;
}

hipError_t launch_debug_map(int64_t nrow, int32_t nchan, const double *uvw,
                            const std::vector<ChanConst> &cc, const MapGeom &g, int32_t *out,
                            hipStream_t s) {
    for (int32_t b = 0; b < nchan; b += kMaxChanPerUpload) {
        ChanUpload up;
        up.n = std::min<int32_t>(kMaxChanPerUpload, nchan - b);
        up.base = b;
        for (int i = 0; i < up.n; ++i) up.c[i] = cc[b + i];
        int64_t n = nrow * up.n;
        if (n == 0) continue;
        hipLaunchKernelGGL(k_debug_map, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           nrow, nchan, uvw, up, g, out);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sort keys.  Fields from most to least significant: plane, A-term group,
// w-plane, conj, p_v, p_u, [baseline, channel when a pointing phasor is
// applied], o_v, o_u.  Keys of dropped or skipped pairs are all ones.
__device__ __forceinline__ void put(unsigned __int128 &key, uint32_t v, int bits) {
    if (bits) key = (key << bits) | (unsigned __int128)v;
}

__global__ void k_plan_keys(int64_t nrow, int32_t nchan, const double *uvw,
                            const ChanConst *cc, MapGeom g, KeyLayout kl,
                            const int32_t *ant1, const int32_t *ant2, int32_t nant,
                            uint64_t *keys, int32_t *vals, unsigned long long *n_kept) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool kept = false;
    if (i < nrow * nchan) {
        int64_t r = i / nchan;
        int32_t c = (int32_t)(i - r * nchan);
        ChanConst ch = cc[c];
        uint64_t key = ~0ull;
        int32_t val = (int32_t)i;
        if (ch.plane < 0) {
            val |= (1 << 30);
        } else {
            Map m = map_sample(uvw[3 * r], uvw[3 * r + 1], uvw[3 * r + 2], ch, g);
            if (m.keep) {
                unsigned __int128 k128 = 0;
                put(k128, (uint32_t)ch.plane, kl.b_plane);
                put(k128, (uint32_t)ch.fg, kl.b_fg);
                put(k128, (uint32_t)m.k, kl.b_k);
                put(k128, (uint32_t)m.conj, kl.b_conj);
                put(k128, (uint32_t)m.pv, kl.b_pv);
                put(k128, (uint32_t)m.pu, kl.b_pu);
                if (kl.b_bl) put(k128, (uint32_t)(ant1[r] * nant + ant2[r]), kl.b_bl);
                if (kl.b_ch) put(k128, (uint32_t)c, kl.b_ch);
                put(k128, (uint32_t)(m.ov + (g.O >> 1)), kl.b_o);
                put(k128, (uint32_t)(m.ou + (g.O >> 1)), kl.b_o);
                key = (uint64_t)(k128 >> kl.shift);
                kept = true;
            }
        }
        keys[i] = key;
        vals[i] = val;
    }
    // one atomic per wavefront
    unsigned long long b = __ballot(kept);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(n_kept, (unsigned long long)__popcll(b));
}

__global__ void k_group_flags(const uint64_t *keys, int64_t n_kept, int32_t merged,
                              int32_t *flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_kept) return;
    flags[i] = (!merged || i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

__device__ __forceinline__ double airy_power(double x) {
    if (x == 0.0) return 1.0;
    double b = 2.0 * j1(x) / x;
    return b * b;
}

__global__ void k_group_meta(const int32_t *vals, const int32_t *flags, const int32_t *gidx,
                             int64_t n_kept, int32_t nchan, const double *uvw,
                             const ChanConst *cc, MapGeom g, CFView cf,
                             const int32_t *ant1, const int32_t *ant2,
                             const double *ant_dlm, double du_dl, double dv_dm,
                             int32_t *group_start, GroupMeta *groups, int64_t *geo) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_kept || !flags[i]) return;
    int32_t gi = gidx[i];
    group_start[gi] = (int32_t)i;
    int32_t pair = vals[i] & ~(1 << 30);
    int64_t r = pair / nchan;
    int32_t c = pair - (int32_t)r * nchan;
    ChanConst ch = cc[c];
    Map m = map_sample(uvw[3 * r], uvw[3 * r + 1], uvw[3 * r + 2], ch, g);
    GroupMeta gm;
    int32_t h = g.h[m.k];
    int64_t S = 2 * h + 1;
    int64_t no = g.O + 1;
    gm.cf_off = cf.plane_off[(int64_t)ch.fg * g.n_w + m.k] +
                ((int64_t)(m.ov + (g.O >> 1)) * no + (m.ou + (g.O >> 1))) * S * S;
    gm.cell = ((int64_t)ch.plane * g.npol) * (int64_t)g.ny * g.nx + (int64_t)m.pv * g.nx + m.pu;
    gm.pu = m.pu;
    gm.pv = m.pv;
    gm.k = m.k;
    gm.conj = m.conj;
    gm.ou = m.ou;
    gm.ov = m.ov;
    gm.plane = ch.plane;
    gm.fg = ch.fg;
    gm.h = h;
    gm.sc = cf.scale[(int64_t)ch.fg * g.n_w + m.k];
    gm.f = 1.0;
    gm.bu = 0.0;
    gm.bv = 0.0;
    if (ant1) {
        int32_t a1 = ant1[r], a2 = ant2[r];
        double l1 = ant_dlm[2 * a1], m1 = ant_dlm[2 * a1 + 1];
        double l2 = ant_dlm[2 * a2], m2 = ant_dlm[2 * a2 + 1];
        double dl = 0.5 * (l1 + l2), dm = 0.5 * (m1 + m2);
        double ddl = l1 - l2, ddm = m1 - m2;
        double dist = sqrt(ddl * ddl + ddm * ddm);
        gm.f = airy_power(ch.fscale * 0.5 * dist);
        gm.bu = (du_dl * dl) / (double)g.O;
        gm.bv = (dv_dm * dm) / (double)g.O;
    }
    groups[gi] = gm;
    geo[gi] = (int64_t)(uint16_t)m.pu | ((int64_t)(uint16_t)m.pv << 16) |
              ((int64_t)(uint16_t)(int16_t)m.ou << 32) | ((int64_t)(uint16_t)(int16_t)m.ov << 48);
}

// The exclusive scan counts a group's own start for every later pair of the
// group; turn it into the group index of every sorted position.
__global__ void k_group_index(int32_t *gidx, const int32_t *flags, int64_t n_kept) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_kept) gidx[i] += flags[i] - 1;
}

__global__ void k_group_end(int32_t *group_start, int64_t n_groups, int64_t n_kept) {
    if (threadIdx.x == 0) group_start[n_groups] = (int32_t)n_kept;
}

// ---- tiles of the gridder ----------------------------------------------------
// Each group's footprint is cut by the 32 x 32 cell tiles it overlaps; the
// (tile, group) pairs are sorted by tile and split into chunks of at most
// `per` pairs, one workgroup each.
__device__ __forceinline__ void tile_span(const GroupMeta &gm, int h, int &tx0, int &tx1,
                                          int &ty0, int &ty1) {
    tx0 = (gm.pu - h) / kTile;
    tx1 = (gm.pu + h) / kTile;
    ty0 = (gm.pv - h) / kTile;
    ty1 = (gm.pv + h) / kTile;
}

__global__ void k_tile_count(const GroupMeta *groups, int64_t n_groups, const int32_t *h,
                             int32_t *counts) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_groups) return;
    GroupMeta gm = groups[i];
    int tx0, tx1, ty0, ty1;
    tile_span(gm, h[gm.k], tx0, tx1, ty0, ty1);
    counts[i] = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
}

__global__ void k_tile_fill(const GroupMeta *groups, int64_t n_groups, const int32_t *h,
                            const int32_t *off, int32_t ntx, int32_t nty, uint32_t *keys,
                            int32_t *vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_groups) return;
    GroupMeta gm = groups[i];
    int tx0, tx1, ty0, ty1;
    tile_span(gm, h[gm.k], tx0, tx1, ty0, ty1);
    int32_t o = off[i];
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) {
            keys[o] = (uint32_t)(((int64_t)gm.plane * nty + ty) * ntx + tx);
            vals[o] = (int32_t)i;
            ++o;
        }
}

// Work of a (tile, group) pair: the cells its footprint covers in the tile.
__global__ void k_pair_cost(const uint32_t *keys, const int32_t *tp_group,
                            const GroupMeta *groups, const int32_t *h, int32_t ntx,
                            int32_t nty, int64_t n, int32_t *cost) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t key = keys[i];
    const int tx = (int)(key % (uint32_t)ntx);
    const int ty = (int)((key / (uint32_t)ntx) % (uint32_t)nty);
    const GroupMeta gm = groups[tp_group[i]];
    const int hh = h[gm.k];
    const int cx = min(gm.pu + hh + 1, (tx + 1) * kTile) - max(gm.pu - hh, tx * kTile);
    const int cy = min(gm.pv + hh + 1, (ty + 1) * kTile) - max(gm.pv - hh, ty * kTile);
    cost[i] = max(cx, 0) * max(cy, 0);
}

// Chunk heads: the first thread of each tile's run of (tile, group) pairs
// (keys sorted by tile) walks the run and opens a new chunk when the current
// one holds `per` pairs or its pairs cover more than `cmax` cells in all, so
// that no workgroup of the gridder gets far more work than the others.  A
// tile that fits one chunk is owned exclusively.
__global__ void k_chunk_flags(const uint32_t *keys, const int32_t *cost, int64_t n,
                              int32_t per, int32_t cmax, int32_t *flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || (i > 0 && keys[i] == keys[i - 1])) return;
    const uint32_t k = keys[i];
    int count = 0, work = 0;
    for (int64_t j = i; j < n && keys[j] == k; ++j) {
        const int c = cost[j];
        const bool head = count == 0 || count == per || work + c > cmax;
        if (head && count > 0) count = work = 0;
        flags[j] = head ? 1 : 0;
        ++count;
        work += c;
    }
}

__global__ void k_chunk_build(const uint32_t *keys, const int32_t *flags, const int32_t *cidx,
                              int64_t n, int32_t *chunk_start, int32_t *chunk_tile) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flags[i]) return;
    int32_t c = cidx[i];
    chunk_start[c] = (int32_t)i;
    chunk_tile[c] = (int32_t)keys[i];
}

// A chunk that holds all of its tile's pairs owns the tile: it may update
// the grid with plain loads and stores instead of atomics.
__global__ void k_chunk_excl(const uint32_t *keys, int32_t *chunk_start, int64_t n_chunks,
                             int64_t n, int32_t *chunk_excl) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_chunks) return;
    int64_t s = chunk_start[c];
    int64_t e = (c + 1 < n_chunks) ? chunk_start[c + 1] : n;
    bool first = (s == 0) || keys[s - 1] != keys[s];
    bool last = (e == n) || keys[e] != keys[e - 1];
    chunk_excl[c] = (first && last) ? 1 : 0;
}

// Work estimate of each chunk (one wavefront per chunk): the footprint
// cells of its pairs inside the tile, complemented so that an ascending
// sort puts the largest first; the chunk ids ride along.
__global__ __launch_bounds__(256) void k_chunk_cost(const int32_t *chunk_start,
                                                    const int32_t *pair_cost, int64_t n_chunks,
                                                    uint32_t *key, int32_t *id) {
    const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (c >= n_chunks) return;
    const int32_t s0 = chunk_start[c], n = chunk_start[c + 1] - s0;
    uint32_t w = 0;
    for (int i = lane; i < n; i += 64) w += (uint32_t)pair_cost[s0 + i];
    for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off);
    if (lane == 0) {
        key[c] = ~w;
        id[c] = (int32_t)c;
    }
}

// Table plane of each chunk (that of its first pair; a tile's pairs follow
// the group order, whose keys put the frequency group and w-plane first, so
// a chunk rarely spans two planes); the chunk ids ride along.
__global__ void k_chunk_plane(const int32_t *chunk_start, const int32_t *tp_group,
                              const GroupMeta *groups, int32_t n_w, int64_t n_chunks,
                              uint32_t *key, int32_t *id) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_chunks) return;
    const GroupMeta &g = groups[tp_group[chunk_start[c]]];
    key[c] = (uint32_t)(g.fg * n_w + g.k);
    id[c] = (int32_t)c;
}

__global__ void k_chunk_end(int32_t *chunk_start, int64_t n_chunks, int64_t n) {
    if (threadIdx.x == 0) chunk_start[n_chunks] = (int32_t)n;
}

// Tile ownership: 1 when one exclusive chunk holds all of the tile's pairs,
// 2 when several chunks share it (tile_state is zeroed beforehand; the
// chunks of a shared tile all store the same value).
__global__ void k_tile_state(const int32_t *chunk_tile, const int32_t *chunk_excl,
                             int64_t n_chunks, int32_t *tile_state) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_chunks) return;
    tile_state[chunk_tile[c]] = chunk_excl[c] ? 1 : 2;
}

// Compact list of the shared tiles (any order).
__global__ void k_shared_list(const int32_t *tile_state, int64_t n_tiles, int32_t *list,
                              int32_t *count) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles || tile_state[t] != 2) return;
    list[atomicAdd(count, 1)] = (int32_t)t;
}

// Single-run groups: with a period L, a group whose pairs are p, p + L,
// p + 2 L, ... (one unbroken stretch of one track) is summed completely by
// the presum lane that walks that track, which may then store the sum
// without an atomic.  single[g] starts at 1 and is cleared by any gap.
__global__ void k_single_init(int32_t *single, int64_t n_groups, int32_t value) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n_groups) single[g] = value;
}

__global__ void k_single_gaps(const int32_t *order, const int32_t *gidx, int64_t n_kept,
                              int64_t period, int32_t *single) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 1 || i >= n_kept || gidx[i] != gidx[i - 1]) return;
    if ((int64_t)order[i] - order[i - 1] != period) single[gidx[i]] = 0;
}

// One-member groups (bit 1 of single[g]; the presum stores their sums, which
// never need a cleared start) and the list of the other groups, which the
// presum may add to with atomics (any order).
__global__ void k_group_kinds(const int32_t *group_start, int64_t n_groups, int32_t *single,
                              int32_t *multi, int32_t *count) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_groups) return;
    if (group_start[g + 1] - group_start[g] == 1) single[g] |= 2;
    else multi[atomicAdd(count, 1)] = (int32_t)g;
}

// First (tile, group) pair of every tile in the tile-sorted pair list
// (keys), by binary search; tile_tp[n_tiles] = n.
__global__ void k_tile_ranges(const uint32_t *keys, int64_t n, int64_t n_tiles,
                              int32_t *tile_tp) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > n_tiles) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)keys[mid] < t) lo = mid + 1; else hi = mid;
    }
    tile_tp[t] = (int32_t)lo;
}

// Parts of the separable gridder: a tile's (tile, group) pairs in pieces of
// at most kSepPart, so that no workgroup is left with a tile many times
// heavier than the rest.  Keys sort the tiles by pair count, most first.
__global__ void k_sep_count(const int32_t *tile_tp, int64_t n_tiles, uint32_t *key,
                            int32_t *tile) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    key[t] = ~(uint32_t)(tile_tp[t + 1] - tile_tp[t]);
    tile[t] = (int32_t)t;
}

__global__ void k_sep_nparts(const int32_t *tile_tp, const int32_t *tile, int64_t n_tiles,
                             int32_t *nparts) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_tiles) return;
    const int32_t t = tile[i];
    const int32_t n = tile_tp[t + 1] - tile_tp[t];
    nparts[i] = (n + kSepPart - 1) / kSepPart;
}

__global__ void k_sep_fill(const int32_t *tile_tp, const int32_t *tile, const int32_t *nparts,
                           const int32_t *first, int64_t n_tiles, int4 *part, int32_t *shared,
                           int32_t *n_shared) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_tiles) return;
    const int32_t t = tile[i], np = nparts[i];
    if (np == 0) return;
    const int32_t b0 = tile_tp[t], b1 = tile_tp[t + 1];
    // equal pieces, the last one shorter by the remainder
    const int32_t len = (b1 - b0 + np - 1) / np;
    for (int q = 0; q < np; ++q)
        part[first[i] + q] = make_int4(t, b0 + q * len, min(b1, b0 + (q + 1) * len), np > 1);
    if (np > 1) shared[atomicAdd(n_shared, 1)] = t;
}

// Group of every pair in natural (row, channel) order: >= 0 kept (bit
// kSingleRun set for a single-run group, kSingleton for a one-member
// group), -1 dropped, -2 skipped channel.
__global__ void k_pair_group(const int32_t *order, const int32_t *gidx, const int32_t *single,
                             int64_t n_kept, int64_t n_pairs, int32_t *pair_group) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pairs) return;
    int32_t v = order[i];
    int32_t pair = v & ~(1 << 30);
    int32_t out = ((v >> 30) & 1) ? -2 : -1;
    if (i < n_kept) {
        const int32_t g = gidx[i];
        const int32_t k = single ? single[g] : 0;
        out = g | ((k & 1) ? kSingleRun : 0) | ((k & 2) ? kSingleton : 0);
    }
    pair_group[pair] = out;
}

// Row period: the smallest r for which rows i and i + r have nearly the same
// (u, v, w) for all of the first 64 rows (the next sample of the same
// baseline in time-major data).  Only the work order of the presum and
// expand kernels depends on it, never a result.
__global__ void k_row_period(const double *uvw, int64_t nrow, int32_t rmax, int32_t *best) {
    int32_t r = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (r > rmax) return;
    int64_t nchk = nrow - r < 64 ? nrow - r : 64;
    if (nchk < 4) return;
    for (int64_t i = 0; i < nchk; ++i) {
        double a0 = uvw[3 * i], a1 = uvw[3 * i + 1], a2 = uvw[3 * i + 2];
        double b0 = uvw[3 * (i + r)], b1 = uvw[3 * (i + r) + 1], b2 = uvw[3 * (i + r) + 2];
        double d = fabs(a0 - b0) + fabs(a1 - b1) + fabs(a2 - b2);
        double s = fabs(a0) + fabs(a1) + fabs(a2);
        if (!(d <= 1e-2 * s + 1e-3)) return;
    }
    atomicMin(best, r);
}

__global__ void k_taps(const GroupMeta *groups, int64_t n_groups, const int32_t *h,
                       unsigned long long *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long t = 0;
    if (i < n_groups) {
        int64_t S = 2 * h[groups[i].k] + 1;
        t = (unsigned long long)(S * S);
    }
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if ((threadIdx.x & 63) == 0 && t) atomicAdd(out, t);
}

// ---------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t sort_temp_bytes(int64_t n, int64_t n_tp) {
    size_t bytes = 0, b2 = 0, sb = 0, sb2 = 0;
    rocprim::radix_sort_pairs((void *)nullptr, bytes, (uint64_t *)nullptr,
                              (uint64_t *)nullptr, (int32_t *)nullptr, (int32_t *)nullptr,
                              (size_t)n, 0, 64);
    rocprim::radix_sort_pairs((void *)nullptr, b2, (uint32_t *)nullptr,
                              (uint32_t *)nullptr, (int32_t *)nullptr, (int32_t *)nullptr,
                              (size_t)n_tp, 0, 32);
    rocprim::exclusive_scan((void *)nullptr, sb, (int32_t *)nullptr, (int32_t *)nullptr,
                            (int32_t)0, (size_t)n, rocprim::plus<int32_t>());
    rocprim::exclusive_scan((void *)nullptr, sb2, (int32_t *)nullptr, (int32_t *)nullptr,
                            (int32_t)0, (size_t)n_tp, rocprim::plus<int32_t>());
    return std::max(std::max(bytes, b2), std::max(sb, sb2));
}

int64_t max_tiles_per_group(int32_t h_max) {
    int64_t span = (2 * (int64_t)h_max + kTile - 1) / kTile + 1;
    return span * span;
}

int64_t tile_count(int32_t nx, int32_t ny, int32_t nplane) {
    return (int64_t)nplane * ((nx + kTile - 1) / kTile) * ((ny + kTile - 1) / kTile);
}

PlanLayout plan_layout(int64_t n_pairs, int32_t nchan, int32_t h_max, int64_t n_tiles) {
    PlanLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    int64_t n = std::max<int64_t>(n_pairs, 1);
    int64_t ntp = n * max_tiles_per_group(h_max);
    L.chan = take(sizeof(ChanConst) * (nchan > 0 ? nchan : 1));
    L.order = take(sizeof(int32_t) * n);
    L.gidx = take(sizeof(int32_t) * n);
    L.pair_group = take(sizeof(int32_t) * n);
    L.group_start = take(sizeof(int32_t) * (n + 1));
    L.groups = take(sizeof(GroupMeta) * n);
    L.tp_group = take(sizeof(int32_t) * ntp);
    L.chunk_start = take(sizeof(int32_t) * (ntp + 1));
    L.chunk_tile = take(sizeof(int32_t) * ntp);
    L.chunk_excl = take(sizeof(int32_t) * ntp);
    L.chunk_order = take(sizeof(int32_t) * ntp);
    L.tile_state = take(sizeof(int32_t) * std::max<int64_t>(n_tiles, 1));
    L.shared_tiles = take(sizeof(int32_t) * std::max<int64_t>(n_tiles, 1));
    L.geo = take(sizeof(int64_t) * n);
    L.tile_tp = take(sizeof(int32_t) * (std::max<int64_t>(n_tiles, 1) + 1));
    L.multi = take(sizeof(int32_t) * n);
    const int64_t nt = std::max<int64_t>(n_tiles, 1);
    L.sep_part = take(sizeof(int4) * (nt + ntp / kSepPart + 1));
    L.sep_shared = take(sizeof(int32_t) * nt);
    L.persistent = off;
    // transient (the tile sort of the separable gridder's parts needs
    // n_tiles + 1 entries)
    const int64_t nx_ = std::max(std::max(n, ntp), nt + 1);
    L.keys_a = take(sizeof(uint64_t) * nx_);
    L.keys_b = take(sizeof(uint64_t) * nx_);
    L.vals_a = take(sizeof(int32_t) * nx_);
    L.flags = take(sizeof(int32_t) * nx_);
    L.scan = take(sizeof(int32_t) * nx_);
    L.counter = take(64);
    L.temp = take(sort_temp_bytes(n, std::max(ntp, nt + 1)));
    L.max_tp = ntp;
    L.total = off;
    return L;
}

static inline unsigned blocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t build_plan_device(lr_plan *P, char *buf, const PlanLayout &L, const double *uvw,
                             const ChanConst *d_cc, const MapGeom &g, const KeyLayout &kl,
                             const CFView &cf, const int32_t *ant1, const int32_t *ant2,
                             int32_t nant, const double *ant_dlm, double du_dl,
                             double dv_dm, int32_t per, int32_t cmax, bool lpt, hipStream_t s) {
    hipError_t e;
    int64_t n = P->n_pairs;
    uint64_t *keys_a = (uint64_t *)(buf + L.keys_a), *keys_b = (uint64_t *)(buf + L.keys_b);
    int32_t *vals_a = (int32_t *)(buf + L.vals_a);
    int32_t *order = (int32_t *)(buf + L.order);
    int32_t *flags = (int32_t *)(buf + L.flags);
    int32_t *gidx = (int32_t *)(buf + L.gidx);
    unsigned long long *counter = (unsigned long long *)(buf + L.counter);
    void *temp = buf + L.temp;
    size_t temp_bytes =
        sort_temp_bytes(n, std::max<int64_t>(L.max_tp, tile_count(g.nx, g.ny, g.nplane) + 1));
    P->order = order;
    P->gidx = gidx;
    P->pair_group = (int32_t *)(buf + L.pair_group);
    P->period = 0;
    P->group_start = (int32_t *)(buf + L.group_start);
    P->groups = (GroupMeta *)(buf + L.groups);
    P->tp_group = (int32_t *)(buf + L.tp_group);
    P->chunk_start = (int32_t *)(buf + L.chunk_start);
    P->chunk_tile = (int32_t *)(buf + L.chunk_tile);
    P->chunk_excl = (int32_t *)(buf + L.chunk_excl);
    P->chunk_order = (int32_t *)(buf + L.chunk_order);
    P->tile_state = (int32_t *)(buf + L.tile_state);
    P->n_tiles = tile_count(g.nx, g.ny, g.nplane);
    P->shared_tiles = (int32_t *)(buf + L.shared_tiles);
    P->n_shared = 0;
    P->geo = (int64_t *)(buf + L.geo);
    P->tile_tp = (int32_t *)(buf + L.tile_tp);
    P->multi = (int32_t *)(buf + L.multi);
    P->n_multi = 0;
    P->sep_part = (int4 *)(buf + L.sep_part);
    P->n_sep_parts = 0;
    P->sep_shared = (int32_t *)(buf + L.sep_shared);
    P->n_sep_shared = 0;
    P->cc = d_cc;
    P->n_kept = P->n_groups = P->n_tile_pairs = P->n_chunks = P->taps = 0;
    if ((e = launch_zero(P->tile_state, sizeof(int32_t) * P->n_tiles, s)) != hipSuccess)
        return e;
    if ((e = launch_zero(P->tile_tp, sizeof(int32_t) * (P->n_tiles + 1), s)) != hipSuccess)
        return e;
    if (n == 0) return hipSuccess;

    if ((e = launch_zero(counter, 64, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_plan_keys, dim3(blocks(n, 256)), dim3(256), 0, s, P->nrow, P->nchan,
                       uvw, d_cc, g, kl, ant1, ant2, nant, keys_a, vals_a, counter);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = rocprim::radix_sort_pairs(temp, temp_bytes, keys_a, keys_b, vals_a, order, (size_t)n,
                                  0, kl.end_bit, s);
    if (e != hipSuccess) return e;
    unsigned long long nk = 0;
    if ((e = hipMemcpyAsync(&nk, counter, sizeof nk, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    P->n_kept = (int64_t)nk;
    if (nk == 0) {
        hipLaunchKernelGGL(k_pair_group, dim3(blocks(n, 256)), dim3(256), 0, s, order, gidx,
                           (const int32_t *)nullptr, (int64_t)0, n, P->pair_group);
        return hipGetLastError();
    }

    hipLaunchKernelGGL(k_group_flags, dim3(blocks(nk, 256)), dim3(256), 0, s, keys_b,
                       (int64_t)nk, P->merged, flags);
    e = rocprim::exclusive_scan(temp, temp_bytes, flags, gidx, (int32_t)0, (size_t)nk,
                                rocprim::plus<int32_t>(), s);
    if (e != hipSuccess) return e;
    int32_t tail[2] = {0, 0};
    (void)hipMemcpyAsync(&tail[0], gidx + nk - 1, 4, hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(&tail[1], flags + nk - 1, 4, hipMemcpyDeviceToHost, s);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    P->n_groups = (int64_t)tail[0] + tail[1];
    hipLaunchKernelGGL(k_group_meta, dim3(blocks(nk, 256)), dim3(256), 0, s, order, flags,
                       gidx, (int64_t)nk, P->nchan, uvw, d_cc, g, cf, ant1, ant2, ant_dlm,
                       du_dl, dv_dm, P->group_start, P->groups, P->geo);
    hipLaunchKernelGGL(k_group_end, dim3(1), dim3(64), 0, s, P->group_start, P->n_groups,
                       (int64_t)nk);
    hipLaunchKernelGGL(k_group_index, dim3(blocks(nk, 256)), dim3(256), 0, s, gidx, flags,
                       (int64_t)nk);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    // (tile, group) pairs and chunks of the gridder
    int32_t *scan = (int32_t *)(buf + L.scan);
    uint32_t *tk_a = (uint32_t *)keys_a, *tk_b = (uint32_t *)keys_b;
    int64_t ng = P->n_groups;
    hipLaunchKernelGGL(k_tile_count, dim3(blocks(ng, 256)), dim3(256), 0, s, P->groups, ng,
                       cf.h, flags);
    e = rocprim::exclusive_scan(temp, temp_bytes, flags, scan, (int32_t)0, (size_t)ng,
                                rocprim::plus<int32_t>(), s);
    if (e != hipSuccess) return e;
    (void)hipMemcpyAsync(&tail[0], scan + ng - 1, 4, hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(&tail[1], flags + ng - 1, 4, hipMemcpyDeviceToHost, s);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    int64_t ntp = (int64_t)tail[0] + tail[1];
    if (ntp > L.max_tp) return hipErrorInvalidValue;
    int32_t ntx = (g.nx + kTile - 1) / kTile, nty = (g.ny + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_tile_fill, dim3(blocks(ng, 256)), dim3(256), 0, s, P->groups, ng,
                       cf.h, scan, ntx, nty, tk_a, vals_a);
    int end_bit = 1;
    while (end_bit < 32 && ((int64_t)1 << end_bit) < (int64_t)g.nplane * ntx * nty) ++end_bit;
    e = rocprim::radix_sort_pairs(temp, temp_bytes, tk_a, tk_b, vals_a, P->tp_group,
                                  (size_t)ntp, 0, end_bit, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pair_cost, dim3(blocks(ntp, 256)), dim3(256), 0, s, tk_b,
                       P->tp_group, P->groups, cf.h, ntx, nty, ntp, vals_a);
    hipLaunchKernelGGL(k_chunk_flags, dim3(blocks(ntp, 256)), dim3(256), 0, s, tk_b, vals_a,
                       ntp, per, cmax, flags);
    e = rocprim::exclusive_scan(temp, temp_bytes, flags, scan, (int32_t)0, (size_t)ntp,
                                rocprim::plus<int32_t>(), s);
    if (e != hipSuccess) return e;
    (void)hipMemcpyAsync(&tail[0], scan + ntp - 1, 4, hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(&tail[1], flags + ntp - 1, 4, hipMemcpyDeviceToHost, s);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    int64_t nch = (int64_t)tail[0] + tail[1];
    hipLaunchKernelGGL(k_chunk_build, dim3(blocks(ntp, 256)), dim3(256), 0, s, tk_b, flags,
                       scan, ntp, P->chunk_start, P->chunk_tile);
    hipLaunchKernelGGL(k_chunk_excl, dim3(blocks(nch, 256)), dim3(256), 0, s, tk_b,
                       P->chunk_start, nch, ntp, P->chunk_excl);
    hipLaunchKernelGGL(k_chunk_end, dim3(1), dim3(64), 0, s, P->chunk_start, nch, ntp);
    hipLaunchKernelGGL(k_tile_ranges, dim3(blocks(P->n_tiles + 1, 256)), dim3(256), 0, s, tk_b,
                       ntp, P->n_tiles, P->tile_tp);
    // with a kernel table the last-level cache holds, the gridder launches
    // chunks largest first (a stable sort: ties keep tile order), so the
    // long ones do not trail the launch; with a larger table it launches
    // them plane by plane (tile order within a plane), so the chunks in
    // flight read one plane of the table, which the cache holds, instead
    // of all of them
    if (nch > 0) {
        int end_bits = 32;
        if (lpt) {
            hipLaunchKernelGGL(k_chunk_cost, dim3(blocks(nch * 64, 256)), dim3(256), 0, s,
                               P->chunk_start, vals_a, nch, tk_a, flags);
        } else {
            hipLaunchKernelGGL(k_chunk_plane, dim3(blocks(nch, 256)), dim3(256), 0, s,
                               P->chunk_start, P->tp_group, P->groups, cf.n_w, nch, tk_a, flags);
            end_bits = 1;
            while (end_bits < 32 && ((int64_t)1 << end_bits) < (int64_t)cf.n_fg * cf.n_w)
                ++end_bits;
        }
        e = rocprim::radix_sort_pairs(temp, temp_bytes, tk_a, (uint32_t *)scan, flags,
                                      P->chunk_order, (size_t)nch, 0, end_bits, s);
        if (e != hipSuccess) return e;
    } else {
        P->chunk_order = nullptr;
    }
    hipLaunchKernelGGL(k_tile_state, dim3(blocks(nch, 256)), dim3(256), 0, s, P->chunk_tile,
                       P->chunk_excl, nch, P->tile_state);
    if ((e = launch_zero(counter, 64, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_shared_list, dim3(blocks(P->n_tiles, 256)), dim3(256), 0, s,
                       P->tile_state, P->n_tiles, P->shared_tiles, (int32_t *)counter);
    int32_t n_shared = 0;
    (void)hipMemcpyAsync(&n_shared, counter, 4, hipMemcpyDeviceToHost, s);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    P->n_shared = n_shared;
    if ((e = launch_zero(counter, 64, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_taps, dim3(blocks(ng, 256)), dim3(256), 0, s, P->groups, ng, cf.h,
                       counter);
    unsigned long long taps = 0;
    (void)hipMemcpyAsync(&taps, counter, 8, hipMemcpyDeviceToHost, s);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    P->n_tile_pairs = ntp;
    P->n_chunks = nch;
    P->taps = (int64_t)taps;

    // parts of the separable gridder, tiles with most pairs first
    {
        const int64_t nt = P->n_tiles;
        uint32_t *ck_a = (uint32_t *)keys_a, *ck_b = (uint32_t *)keys_b;
        int32_t *tid_s = (int32_t *)scan;
        hipLaunchKernelGGL(k_sep_count, dim3(blocks(nt, 256)), dim3(256), 0, s, P->tile_tp, nt,
                           ck_a, vals_a);
        e = rocprim::radix_sort_pairs(temp, temp_bytes, ck_a, ck_b, vals_a, tid_s, (size_t)nt,
                                      0, 32, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_sep_nparts, dim3(blocks(nt, 256)), dim3(256), 0, s, P->tile_tp,
                           tid_s, nt, flags);
        int32_t *first = (int32_t *)ck_a;
        e = rocprim::exclusive_scan(temp, temp_bytes, flags, first, (int32_t)0, (size_t)nt,
                                    rocprim::plus<int32_t>(), s);
        if (e != hipSuccess) return e;
        if ((e = launch_zero(counter, 64, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_sep_fill, dim3(blocks(nt, 256)), dim3(256), 0, s, P->tile_tp,
                           tid_s, flags, first, nt, P->sep_part, P->sep_shared,
                           (int32_t *)counter);
        int32_t tl[3] = {0, 0, 0};
        (void)hipMemcpyAsync(&tl[0], first + nt - 1, 4, hipMemcpyDeviceToHost, s);
        (void)hipMemcpyAsync(&tl[1], flags + nt - 1, 4, hipMemcpyDeviceToHost, s);
        (void)hipMemcpyAsync(&tl[2], counter, 4, hipMemcpyDeviceToHost, s);
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        P->n_sep_parts = (int64_t)tl[0] + tl[1];
        P->n_sep_shared = tl[2];
    }

    // the row period of the data, then the natural-order group map
    int32_t rmax = (int32_t)std::min<int64_t>(P->nrow - 1, 1 << 16);
    P->period = 0;
    if (rmax >= 1) {
        int32_t *best = (int32_t *)counter;
        int32_t big = 0x7fffffff;
        if ((e = upload_words(&big, sizeof big, best, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_row_period, dim3(blocks(rmax, 256)), dim3(256), 0, s, uvw,
                           P->nrow, rmax, best);
        int32_t r = big;
        (void)hipMemcpyAsync(&r, best, 4, hipMemcpyDeviceToHost, s);
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        if (r != big) P->period = (int64_t)r * P->nchan;
    }
    // groups that are one unbroken stretch of one track (pairs of another
    // track, or a gap, break the stride L between consecutive members)
    int32_t *single = flags;
    hipLaunchKernelGGL(k_single_init, dim3(blocks(ng, 256)), dim3(256), 0, s, single, ng,
                       P->period > 0 ? 1 : 0);
    if (P->period > 0)
        hipLaunchKernelGGL(k_single_gaps, dim3(blocks(nk, 256)), dim3(256), 0, s, order, gidx,
                           (int64_t)nk, P->period, single);
    if ((e = launch_zero(counter, 64, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_group_kinds, dim3(blocks(ng, 256)), dim3(256), 0, s, P->group_start,
                       ng, single, P->multi, (int32_t *)counter);
    int32_t n_multi = 0;
    (void)hipMemcpyAsync(&n_multi, counter, 4, hipMemcpyDeviceToHost, s);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    P->n_multi = n_multi;
    hipLaunchKernelGGL(k_pair_group, dim3(blocks(n, 256)), dim3(256), 0, s, order, gidx,
                       (const int32_t *)single, (int64_t)nk, n, P->pair_group);
    return hipGetLastError();
}

}  // namespace lr
