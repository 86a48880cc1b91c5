// Host-side launchers of the gfx950 kernels, called by the C ABI layer.
#pragma once

#include <vector>

#include "lr_internal.h"

namespace lr {

// ---- plan (k_plan.hip) -------------------------------------------------------
struct KeyLayout {
    int32_t b_plane, b_fg, b_k, b_conj, b_pv, b_pu, b_bl, b_ch, b_o;
    int32_t shift;     // right shift applied to the full key
    int32_t end_bit;   // significant bits of the final key
};

struct PlanLayout {
    size_t chan, order, gidx, pair_group, group_start, groups, tp_group, chunk_start, chunk_tile,
        chunk_excl, chunk_order, tile_state, shared_tiles, geo, tile_tp, multi, sep_part,
        sep_shared, persistent;
    size_t keys_a, keys_b, vals_a, flags, scan, counter, temp;
    int64_t max_tp;
    size_t total;
};

hipError_t upload_chan(const std::vector<ChanConst> &cc, ChanConst *d, hipStream_t s);
hipError_t upload_words(const void *src, size_t bytes, void *d, hipStream_t s);
hipError_t launch_debug_map(int64_t nrow, int32_t nchan, const double *uvw,
                            const std::vector<ChanConst> &cc, const MapGeom &g, int32_t *out,
                            hipStream_t s);
size_t sort_temp_bytes(int64_t n, int64_t n_tp);
int64_t max_tiles_per_group(int32_t h_max);
PlanLayout plan_layout(int64_t n_pairs, int32_t nchan, int32_t h_max, int64_t n_tiles);
int64_t tile_count(int32_t nx, int32_t ny, int32_t nplane);
hipError_t build_plan_device(lr_plan *P, char *buf, const PlanLayout &L, const double *uvw,
                             const ChanConst *d_cc, const MapGeom &g, const KeyLayout &kl,
                             const CFView &cf, const int32_t *ant1, const int32_t *ant2,
                             int32_t nant, const double *ant_dlm, double du_dl,
                             double dv_dm, int32_t per, int32_t cmax, bool lpt, hipStream_t s);

// ---- CF build (k_cf.hip) -----------------------------------------------------
struct CFBuildArgs {
    int32_t M, O, nx, ny, terms;
    double cell_l, cell_m, c_ps, dish_m;
    int32_t pol_beam, kind;     // polarised beam: the Mueller kind of the screen
    double eta, kappa;          // beam ellipticity and leakage
};
size_t cf_work_bytes(int32_t M, int32_t O, int32_t h_max);
hipError_t launch_cf_build(const lr_cf *cf, const CFBuildArgs &a, void *work, hipStream_t s);

// ---- hot path (k_grid.hip) ---------------------------------------------------
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);

struct VisArgs {
    const void *vis;
    const void *weight;
    int32_t npol;
    int32_t unit_vis;      // PSF: visibilities taken as 1
};

// presum: per group A[g][pol] += sum W V over its pairs (A zeroed by
// launch_grid_setup); counters and sumwt
hipError_t launch_presum(const lr_plan *P, const VisArgs &v, int precision, void *A,
                         double *sumwt, int64_t *counters, int32_t nplane, hipStream_t s);
hipError_t launch_counts(const lr_plan *P, const void *weight, int precision, int32_t npol,
                         double *sumwt, int64_t *counters, int32_t nplane, hipStream_t s);
// mode: GRID_ADD (grid +=), GRID_PSF (grid += half the mirror pair), GRID_SET
// (grid =, every cell written; zero_tiles must have run on the same stream)
enum { GRID_ADD = 0, GRID_PSF = 1, GRID_SET = 2 };
// det: deterministic order (one workgroup per tile, no atomic flushes; not
// for GRID_PSF)
// mix (Mueller passes; 0 = none): bit q * npol + p set when correlation q's
// group sums go into grid pol p in this pass.
hipError_t launch_grid(const lr_plan *P, const CFView &cf, const void *A, void *grid,
                       int precision, int32_t npol, int32_t nx, int32_t ny, int32_t mode,
                       bool det, uint32_t mix, hipStream_t s);
// Whether launch_grid takes the separable small-support gridder (one
// workgroup per tile, every cell written once): then GRID_SET needs no
// clearing of shared tiles beforehand.
bool sep_gridder(const lr_plan *P, const CFView &cf, int32_t mode, bool det);
// The separable gridder's launch (k_sep.hip), when sep_gridder() chose it.
hipError_t launch_grid_sep(const lr_plan *P, const CFView &cf, const void *A, void *grid,
                           int precision, int32_t npol, int32_t nx, int32_t ny, bool set,
                           hipStream_t s);
// Set-up of a gridding call, one launch: zero the group sums A (a_bytes)
// and, when given, sumwt and counters; under GRID_SET also the tiles that
// several chunks share (they are then added to atomically).
// sep: the separable gridder follows, whose shared tiles (split into
// several parts) are the ones cleared under GRID_SET.
hipError_t launch_grid_setup(const lr_plan *P, void *A, size_t a_bytes, double *sumwt,
                             size_t sumwt_bytes, int64_t *counters, void *grid,
                             int precision, int32_t npol, int32_t nx, int32_t ny, bool set,
                             bool sep, hipStream_t s);
// h_max: widest half-width of the table (small supports take the
// four-groups-per-wavefront degridder)
// mix (Mueller passes; 0 = none): bit q * npol + p set when grid pol p's
// gather adds into correlation q; accum adds to Vg instead of writing it.
hipError_t launch_degrid(const lr_plan *P, const CFView &cf, const void *grid, void *Vg,
                         int precision, int32_t npol, int32_t nx, int32_t ny, int32_t h_max,
                         uint32_t mix, bool accum, hipStream_t s);
hipError_t launch_expand(const lr_plan *P, const void *Vg, void *vis, const void *weight,
                         int precision, int32_t npol, hipStream_t s);

// ---- image plane (k_image.hip) ------------------------------------------------
hipError_t launch_gcf(const CFView &cf, int64_t plane_base, int32_t h, float sc, int32_t n,
                      double2 *out, hipStream_t s);
hipError_t launch_normalize(const void *img, const double *gx, const double *gy,
                            const double *sumwt, int32_t nx, int32_t ny, int64_t n_planes,
                            int precision, void *out, hipStream_t s);

hipError_t launch_normalize_pb(const void *img, const double *gx, const double *gy,
                               const double *sumwt, const double *pb, double pb_min,
                               int32_t nx, int32_t ny, int64_t n_planes, int precision,
                               void *out, hipStream_t s);
// PS taper at n image pixels (k_cf.hip); weight image of A-projection
hipError_t launch_ps_taper(double c, int use_ps, int32_t n, double *out, hipStream_t s);
hipError_t launch_pb_image(const lr_cf *cf, const double *w, double *out, hipStream_t s);

// ---- minor cycle (k_hogbom.hip) -------------------------------------------------
constexpr int kHogbomBlocks = 1024;      // workgroups of the peak search
size_t hogbom_work_bytes(int32_t nx, int32_t ny);
hipError_t launch_hogbom(void *res, const void *psf, void *model, int32_t nx, int32_t ny,
                         int precision, double gain, double threshold, int32_t niter,
                         void *work, int32_t *iters, hipStream_t s);

// ---- calibration (k_cal.hip) ----------------------------------------------------
struct CalVavg {
    const void *obs, *mod, *weight;
    const int32_t *ant1, *ant2, *row_sol, *chan_sol;
    int64_t nrow;
    int32_t nchan, npol, nant, n_tsol, n_fsol, rows_per_step, precision;
    double *X, *w;
};
hipError_t launch_cal_vavg(const CalVavg &c, hipStream_t s);
hipError_t launch_cal_solve(const double *X, const double *w, int32_t nant, int64_t n_prob,
                            double alpha, double delta, int32_t max_iter, double *g,
                            int32_t *iterations, double *change, hipStream_t s);

// ---- mosaic (k_mosaic.hip) ---------------------------------------------------------
hipError_t launch_rephase(void *vis, const double *uvw, const double *freq_hz,
                          const int32_t *field, const double *field_dlm, int64_t nrow,
                          int32_t nchan, int32_t npol, int32_t nfield, int precision,
                          int32_t direction, hipStream_t s);

// ---- deterministic gridding sums (k_grid.hip) ---------------------------------
// Row blocks per channel of the deterministic sums of weights; the partials
// take nchan * kDetRowBlocks * npol doubles of workspace.
constexpr int kDetRowBlocks = 64;
// Members per segment of the deterministic group sums; the pieces of groups
// that cross segment edges take 2 * npol complex values per segment.
constexpr int kDetSeg = 256;
// Group sums in a fixed order, stored (no clear needed): with a row period
// the column presum stores the groups it holds whole and flags them in
// done[n_groups]; every other group is summed over fixed segments of the
// plan's sorted order, pieces in part[ceil(n_kept / kDetSeg)][2][npol].
// Adds the sample counts to counters (if not null).
hipError_t launch_presum_det(const lr_plan *P, const VisArgs &v, int precision, void *A,
                             uint8_t *done, void *part, int64_t *counters, hipStream_t s);
// sumwt[plane][pol] += sum of kept weights, in a fixed order.
hipError_t launch_sumwt_det(const lr_plan *P, const void *weight, int precision, int32_t npol,
                            int32_t nplane, double *part, double *sumwt, hipStream_t s);

}  // namespace lr
