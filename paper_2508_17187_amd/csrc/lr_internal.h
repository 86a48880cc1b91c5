// Internal declarations of the gfx950 gridding library: handle structs,
// device parameter blocks and the per-sample index map shared by the
// kernels.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lr.h"

namespace lr {

constexpr double kCLight = 299792458.0;
constexpr int kMaxChanPerUpload = 48;
constexpr int kTile = 32;          // gridder tile side (cells)
constexpr int kChunkMax = 64;      // most (tile, group) pairs per gridder workgroup
// most footprint cells per workgroup: a pair covers at most one tile, so
// this cap binds only below kChunkMax pairs of whole-tile footprints (a cap
// of 32 tiles cost the large A+W image 7% of its gridder time in extra
// atomic flushes, with no gain on 2048^2 grids)
constexpr int kChunkCells = kChunkMax * kTile * kTile;
constexpr int32_t kSingleRun = 1 << 30;   // pair_group flag: the group is one stretch of a track
constexpr int32_t kSingleton = 1 << 29;   // pair_group flag: the group has one member
constexpr int32_t kGroupFlags = kSingleRun | kSingleton;
constexpr int kSepPart = 4096;     // most (tile, group) pairs per workgroup of the separable gridder

// ---------------------------------------------------------------------------
// Per-channel constants formed on the host in FP64 (no contraction).
struct ChanConst {
    double kx, ky, kw;      // scale to 1/O-cell units and to w-plane units
    double fscale;          // pi * D * nu / c, argument scale of the loss term
    int32_t plane, fg;      // output plane (< 0: skipped), A-term group
    int32_t pad0, pad1;
};

// Geometry the index map needs, passed by value to kernels.
struct MapGeom {
    int32_t nx, ny, O, n_w;
    int32_t psf, npol, nplane, nchan;
    double ox, oy, limx, limy;
    const int32_t *h;       // device [n_w]
};

struct Map {
    int32_t pu, pv, ou, ov, k, conj, keep;
};

// The index map of one (row, channel).  Exactly one rounding per coordinate
// (fma), then floor and integer arithmetic only: bit-exact with a correct
// host implementation of the same definition.
__device__ __forceinline__ Map map_sample(double u, double v, double w, const ChanConst &cc,
                                          const MapGeom &g) {
    Map m;
    m.pu = m.pv = m.ou = m.ov = m.k = m.conj = m.keep = 0;
    double X = fma(u, cc.kx, g.ox);
    double Y = fma(v, cc.ky, g.oy);
    if (!(X >= 0.0 && X < g.limx) || !(Y >= 0.0 && Y < g.limy)) return m;
    int32_t qx = (int32_t)floor(X);
    int32_t qy = (int32_t)floor(Y);
    int32_t half = g.O >> 1;
    // q + O/2 >= 0 here, so C division is floor division
    int32_t px = (qx + half) / g.O;
    int32_t py = (qy + half) / g.O;
    m.pu = px;
    m.pv = py;
    m.ou = qx - px * g.O;
    m.ov = qy - py * g.O;
    double kk = floor(fma(fabs(w), cc.kw, 0.5));
    if (!(kk <= (double)(g.n_w - 1))) return m;
    m.k = (int32_t)kk;
    m.conj = (g.n_w > 1 && w < 0.0) ? 1 : 0;
    int32_t h = g.h[m.k];
    int32_t lo = g.psf ? 1 : 0;
    if (px - h < lo || px + h > g.nx - 1) return m;
    if (py - h < lo || py + h > g.ny - 1) return m;
    m.keep = 1;
    return m;
}

// ---------------------------------------------------------------------------
// One group: kept (row, channel) pairs with identical plane, kernel and
// footprint (and, with a pointing phasor, identical baseline and channel).
struct GroupMeta {
    int64_t cf_off;         // element offset of the S x S sub-kernel in the table
    int64_t cell;           // P*npol*ny*nx + p_v*nx + p_u (pol 0)
    int32_t pu, pv;
    int32_t k, conj;        // w-plane, conjugate flag
    int32_t ou, ov;         // oversampling offsets in [-O/2, O/2)
    int32_t plane, fg;
    int32_t h;              // half-width of the w-plane's support
    float sc;               // 2^-e of the CF plane (1 for f32 / f64 storage)
    double f;               // pointing loss factor (1 without phasor)
    double bu, bv;          // phasor slopes du*dl/O and dv*dm/O (0 without)
};

// Device view of a CF table.
struct CFView {
    const void *table;
    const int64_t *plane_off;   // [n_fg*n_w] element offsets
    const float *scale;         // [n_fg*n_w] 2^-e (1 for f32 / f64)
    const int32_t *h;           // [n_w]
    int32_t O, n_w, n_fg, storage;
    int32_t real;               // every value real (no A term, no w-dependence)
    int32_t h0;                 // half-width of w-plane 0
    int64_t off0;               // element offset of plane (0, 0)
};

}  // namespace lr

// ---------------------------------------------------------------------------
// Host handles (opaque to callers).
struct lr_cf {
    lr_cf_spec spec;
    std::vector<double> fg_hz;
    lr_grid_spec grid;
    int32_t M;
    std::vector<int32_t> h;
    std::vector<int64_t> plane_off;     // element offsets (kind 0)
    int64_t n_elems;                    // elements of every kind
    int32_t n_kind;                     // Mueller kinds held (1: scalar beam)
    int64_t kind_elems;                 // elements per kind
    int32_t kind_of[16];                // kind of M[q][p] (q * 4 + p), -1 none
    size_t elem_bytes;
    size_t header_bytes, total_bytes;
    char *blob;                         // device
    int32_t *d_h;
    int64_t *d_plane_off;
    int32_t *d_exp;
    float *d_scale;
    void *d_table;
};

struct lr_plan {
    // what it was built for
    const lr_cf *cf;
    int64_t nrow;
    int32_t nchan, npol, psf, po, merged;
    std::vector<double> freq;
    std::vector<int32_t> chan_plane, chan_fg;
    // counts
    int64_t n_pairs, n_kept, n_groups, n_tile_pairs, n_chunks, taps;
    // device arrays inside the caller's buffer
    int32_t *order;            // [n_pairs] pair ids; kept (sorted) first; bit 30 set = skipped channel
    int32_t *gidx;             // [n_kept] group of each sorted kept pair
    int32_t *pair_group;       // [n_pairs] group of each pair in natural order (-1 dropped,
                               // -2 skipped; kSingleRun set for single-run groups,
                               // kSingleton for one-member groups)
    int64_t period;            // pairs between consecutive samples of one track (0: unknown)
    int32_t *group_start;      // [n_groups + 1]
    lr::GroupMeta *groups;     // [n_groups]
    int32_t *tp_group;         // [n_tile_pairs] group of each (tile, group) pair, by tile
    int32_t *chunk_start;      // [n_chunks + 1] first pair of each gridder chunk
    int32_t *chunk_tile;       // [n_chunks] tile id: (plane * nty + ty) * ntx + tx
    int32_t *chunk_excl;       // [n_chunks] 1 when the chunk holds all pairs of its tile
    int32_t *chunk_order;      // [n_chunks] launch order: by estimated work, largest
                               // first, for kernel tables the last-level cache holds;
                               // plane by plane for larger ones (null: no chunks)
    int32_t *tile_state;       // [n_tiles] 0 no pairs, 1 one exclusive chunk, 2 several chunks
    int64_t n_tiles;           // nplane * nty * ntx
    int32_t *shared_tiles;     // [n_shared] ids of the tiles in state 2
    int64_t n_shared;
    int64_t *geo;              // [n_groups] (p_u, p_v, o_u, o_v) as int16, p_u lowest
    int32_t *tile_tp;          // [n_tiles + 1] first (tile, group) pair of each tile
    int32_t *multi;            // [n_multi] groups with more than one member
    int64_t n_multi;
    int4 *sep_part;            // [n_sep_parts] (tile, first pair, end pair, several parts)
                               // of the separable gridder, tiles with most pairs first
    int64_t n_sep_parts;
    int32_t *sep_shared;       // [n_sep_shared] tiles split into several parts
    int64_t n_sep_shared;
    const lr::ChanConst *cc;   // [nchan] channel constants (plane of each channel)
    size_t bytes_used;
};
