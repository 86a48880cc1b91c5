/*
 * lr.h -- C ABI of the MI355X (gfx950) convolutional gridding / degridding
 * library.
 *
 * The operations follow the paper's statement of the imaging problem
 * (Bhatnagar et al., "An Algorithm Architecture for Radio Interferometric
 * Data Processing"):
 *   degridding D(c_ij)   Eq. ME-MOD-GRIDDED: model visibilities resampled off
 *                        the regular grid through the kernels c_ij;
 *   gridding G(c_ij)     Eq. IMAGE-MOD: weighted visibilities w_ij V_ij
 *                        accumulated onto the regular grid (the "reverse
 *                        operator" of D);
 *   kernels c_ij         Eq. CIJ and Table AWP-CFSETUP: oversampled PS, A and
 *                        W convolution functions held in a CF cache (the
 *                        PreCompute component), with the per-baseline
 *                        pointing-offset phasor applied on the fly;
 *   summations over t, nu  Eq. ResIm and the OutTransform component: a channel
 *                        map chooses accumulation (continuum) or gather
 *                        (cube planes).
 *
 * Conventions (the paper leaves them open; these are this library's):
 *   - A sample is one (row, channel, polarisation) complex visibility.
 *   - Grid layout [nplane][npol][ny][nx], complex interleaved (re, im), x
 *     fastest.  u = 0 lies at pixel nx/2, v = 0 at ny/2; the uv cell is
 *     du = 1/(nx cell_l).
 *   - Per channel the host forms, in FP64 left to right:
 *       s = nu/c;  kx = ((s nx) cell_l) O;  ky = ((s ny) cell_m) O;
 *       kw = s ((n_w - 1)/w_max) (0 if n_w == 1);  ox = (nx/2) O + 1/2.
 *     Per sample the device forms X = fma(u, kx, ox) (one rounding), drops
 *     the sample unless 0 <= X < nx O, takes q = floor(X), p = floor((q +
 *     O/2)/O), o = q - p O in [-O/2, O/2); the w-plane is
 *     k = floor(fma(|w|, kw, 1/2)) and the kernel is conjugated when w < 0
 *     (n_w > 1).  These integers are bit-exact with the CPU oracle.
 *   - Support of w-plane k: S_k = 2 h_k + 1, h_k = h_min + floor((2 (h_max -
 *     h_min) k + n_w - 1) / (2 (n_w - 1))).  A sample whose footprint
 *     [p - h_k, p + h_k] leaves [0, N-1] (PSF: [1, N-1]) on either axis, or
 *     whose k exceeds n_w - 1, is dropped and counted, never clamped.
 *   - A sample is flagged when its weight is 0 or its channel maps to a
 *     negative plane.  counters[3] = {kept, flagged, dropped} (int64).
 *
 * Memory: every device buffer is caller-owned.  Sizes come from the *_bytes
 * queries.  lr_cf and lr_plan handles are small host objects that describe
 * caller-owned device blobs.  Outputs grid, psf_grid, sumwt and counters
 * are ACCUMULATED (+=), so partitions of the data can be gridded into the
 * same grid; the caller zeroes them.  lr_degrid OVERWRITES vis.
 *
 * Errors: every entry point returns an lr_status; host-side validation runs
 * before anything is enqueued and leaves outputs untouched.  Work is
 * asynchronous on the given stream (NULL = the null stream).  A device
 * fault surfaces as LR_E_DEVICE on a later call or at synchronisation.
 * lr_last_error() gives a thread-local message for the last failure.
 * Calls are re-entrant; concurrent calls must not share outputs or scratch.
 */
#ifndef LR_H
#define LR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *lr_stream;     /* a hipStream_t */

typedef enum {
    LR_OK = 0,
    LR_E_ARG = -1,        /* a malformed descriptor or pointer */
    LR_E_DTYPE = -2,      /* CF storage does not match the precision form */
    LR_E_WORKSPACE = -3,  /* a caller buffer is smaller than required */
    LR_E_CF = -4,         /* the CF blob is not a valid table for this spec */
    LR_E_DEVICE = -5,     /* a HIP runtime error */
    LR_E_RANGE = -6       /* a size beyond the supported range */
} lr_status;

/* Precision forms.  LR_F64: complex128 vis and grid, float64 weights, f64 CF.
 * LR_F32: complex64 vis and grid, float32 weights, f32 CF.  LR_F32_CF16 /
 * LR_F32_CFBF16: as LR_F32 with the CF stored as fp16 / bf16 pairs scaled by
 * 2^e per plane, accumulation in FP32.  In every form the uvw scaling, the
 * index map, the pointing-phasor argument and sumwt are FP64. */
typedef enum { LR_F64 = 0, LR_F32 = 1, LR_F32_CF16 = 2, LR_F32_CFBF16 = 3 } lr_precision;

/* CF terms, Table AWP-CFSETUP: PS = anti-aliasing prolate spheroidal taper,
 * W = W-term, A = antenna aperture (Airy power pattern). */
enum { LR_TERM_PS = 1u, LR_TERM_W = 2u, LR_TERM_A = 4u };

typedef struct {
    int32_t nx, ny;        /* even, 8 .. 16384 */
    int32_t npol;          /* correlations: 1, 2 or 4 */
    int32_t nplane;        /* output planes (cube channels or 1) */
    double cell_l, cell_m; /* image cell, radians */
} lr_grid_spec;

/* Kernel construction (Table AWP-CFSETUP; the CFCache / ConvFunc
 * components).  The screen T(l) T(m) [B] [W_k] is sampled on (M+1)^2 points
 * spanning the image with trapezoid end weights, transformed by a length O M
 * DFT, cropped to S_k x S_k taps for each of the (O+1)^2 offsets
 * o in [-O/2, O/2], divided by M^2 and conjugated. */
typedef struct {
    uint32_t terms;        /* LR_TERM_* bit set, nonzero */
    int32_t oversample;    /* O, even, 2 .. 126 */
    int32_t ps_support;    /* S_ps of the PS taper: c = pi S_ps / 2 */
    int32_t n_w;           /* w-planes, 1 .. 255 */
    double w_max;          /* wavelengths mapped to plane n_w - 1 (n_w > 1) */
    int32_t h_min, h_max;  /* support half-widths, 0 <= h_min <= h_max <= 128 */
    int32_t n_fg;          /* A-term frequency groups, 1 .. 127 */
    const double *fg_hz;   /* host [n_fg]: frequency of each group's A-term */
    double dish_m;         /* Airy dish diameter (A term) */
    int32_t screen_m;      /* M, even; 0 = smallest even >= 2 S_max */
    lr_precision storage;  /* element type of the table */
    /* Sparse Mueller matrix of CFs (the AWP framework's VisResampler holds
     * F M^DD as a 2-D sparse matrix of kernels; M^DD = J (x) J for identical
     * antennas, Eq. ME).  pol_beam = 0: one scalar A term, the Airy power
     * pattern, for every correlation (a diagonal Mueller matrix of one
     * kernel).  pol_beam = 1, 2, 3: a polarised beam for linear feeds
     * (correlations XX, XY, YX, YY, index q = 2 q1 + q2), J = [[E_X, d],
     * [d, E_Y]] with a(x) = 2 J1(x)/x and s = pi dish_m nu_fg / c:
     *   E_X = a(s sqrt((l/(1+eta))^2 + (m/(1-eta))^2)), E_Y: eta -> -eta,
     *   d   = kappa (s l)(s m) a(s rho)   (four-lobed cross-polar leakage),
     * keeping the elements M[q][p] = J[q1][p1] J[q2][p2] of order below
     * pol_beam in d (4, 12 or all 16 elements).  The table then holds the
     * distinct products ("kinds") one after the other: E_X^2, E_Y^2,
     * E_X E_Y, E_X d, E_Y d, d^2 (3, 5 or 6 of them).  Needs LR_TERM_A and
     * npol = 4.  The model is this library's reading: the paper gives no
     * polarised beam.  Zero-initialised fields keep the scalar beam. */
    int32_t pol_beam;          /* 0 .. 3 */
    double beam_ellipticity;   /* eta, |eta| < 0.5 */
    double beam_leakage;       /* kappa, |kappa| <= 10 */
} lr_cf_spec;

typedef struct lr_cf lr_cf;       /* host handle over a caller-owned device blob */
typedef struct lr_plan lr_plan;   /* host handle over a caller-owned device blob */

/* Visibility data.  Device pointers unless noted; uvw, vis and weight must be
 * 16-byte aligned (LR_E_ARG otherwise). */
typedef struct {
    int64_t nrow;
    int32_t nchan, npol, nant;
    const double *uvw;          /* [nrow][3] metres, FP64 */
    const double *freq_hz;      /* host [nchan] */
    const int32_t *chan_plane;  /* host [nchan]: output plane, < 0 = skip */
    const int32_t *chan_fg;     /* host [nchan] A-term group, or NULL = 0 */
    void *vis;                  /* [nrow][nchan][npol] complex128 | complex64 */
    const void *weight;         /* same shape, float64 | float32; 0 = flagged.
                                   lr_degrid accepts NULL (nothing flagged) */
    const int32_t *ant1, *ant2; /* [nrow], or NULL: no pointing phasor */
    const double *ant_dlm;      /* [nant][2] pointing offsets (rad), or NULL */
    const lr_plan *plan;        /* binning from lr_plan_build, or NULL */
} lr_vis;

/* ---- sizes ---------------------------------------------------------------- */

/* Bytes of the device blob lr_cf_build fills (header + table); 0 when the
 * specs are invalid (lr_last_error says why). */
size_t lr_cf_bytes(const lr_cf_spec *spec, const lr_grid_spec *grid);

enum { LR_OP_CF_BUILD = 0, LR_OP_GRID = 1, LR_OP_DEGRID = 2, LR_OP_PSF = 3,
       LR_OP_SUMWT = 4 };

/* Device scratch bytes an operation needs.  For LR_OP_CF_BUILD, vis may be
 * NULL.  For the visibility operations the figure covers a transient plan
 * when vis->plan is NULL.  0 on invalid arguments. */
size_t lr_workspace_bytes(int op, const lr_cf_spec *spec, const lr_grid_spec *grid,
                          const lr_vis *vis, lr_precision precision);

/* ---- convolution functions (PreCompute) ------------------------------------- */

/* Build the CF table for `spec` on `grid` into cf_buf (device, cf_bytes >=
 * lr_cf_bytes) using `work` (device scratch, >= lr_workspace_bytes(
 * LR_OP_CF_BUILD, ...)).  On LR_OK *out receives a host handle; the blob is
 * immutable afterwards and may be shared by concurrent calls.  The handle
 * must be released with lr_cf_free (which does not free cf_buf). */
lr_status lr_cf_build(const lr_cf_spec *spec, const lr_grid_spec *grid, void *cf_buf,
                      size_t cf_bytes, void *work, size_t work_bytes, lr_stream stream,
                      lr_cf **out);

/* Wrap an already built blob (same spec and grid) without recomputing it. */
lr_status lr_cf_attach(const lr_cf_spec *spec, const lr_grid_spec *grid, void *cf_buf,
                       size_t cf_bytes, lr_cf **out);

void lr_cf_free(lr_cf *cf);

/* Per-plane storage exponent e_k (table entries are C * 2^e_k) read back to
 * the host into exps[n_kind * n_fg * n_w] (kind-major); synchronises the
 * stream. */
lr_status lr_cf_scale_exponents(const lr_cf *cf, int32_t *exps, lr_stream stream);

/* Where the table lives in the blob: byte offset of element 0, bytes per
 * complex element (16 f64, 8 f32, 4 fp16/bf16 pair), element count (of
 * every kind), and the element offset of every plane (fg, k) of kind 0 in
 * plane_off[n_fg * n_w] (may be NULL).  The table is laid out [kind][fg][k]
 * [o_v + O/2][o_u + O/2][t_v + h_k][t_u + h_k], o in [-O/2, O/2]; kind
 * kappa starts kappa * n_elems / n_kind elements after kind 0. */
lr_status lr_cf_layout(const lr_cf *cf, size_t *table_offset, size_t *elem_bytes,
                       int64_t *n_elems, int64_t *plane_off);

/* The Mueller kinds of the table: *n_kind (1 for the scalar beam) and, when
 * kind_of is not NULL, kind_of[q * 4 + p] = kind of element M[q][p] or -1
 * (scalar beam: 0 on the diagonal of npol x npol, -1 elsewhere, 16 entries
 * written).  Gridding adds sum_q Ct_qp W_q V_q into pol p; degridding gives
 * V_q = sum_p conj(Ct_qp) grid_p.  Host only. */
lr_status lr_cf_kinds(const lr_cf *cf, int32_t *n_kind, int32_t *kind_of);

/* ---- binning (PreSolvePrep) ------------------------------------------------ */

/* Bytes of the device blob a plan needs for this data. */
size_t lr_plan_bytes(const lr_cf *cf, const lr_vis *vis, int psf);

/* Map every (row, channel), drop what leaves the grid, sort the rest by
 * (plane, CF plane, w-plane, conj, pixel, offset) and merge samples whose
 * kernel and footprint are identical into groups.  The plan depends on uvw,
 * frequencies, channel maps, the CF geometry and (with a pointing phasor)
 * the antenna ids, never on visibilities or weights.  psf != 0 builds the
 * plan for the PSF footprint rule.  Synchronises the stream once (group and
 * task counts come back to the host).  buf must stay alive while the plan
 * is used; release the handle with lr_plan_free. */
lr_status lr_plan_build(const lr_cf *cf, const lr_vis *vis, int psf, void *buf,
                        size_t bytes, lr_stream stream, lr_plan **out);

void lr_plan_free(lr_plan *plan);

/* Bytes a built plan's arrays take at their actual sizes.  lr_plan_build
 * needs a buffer sized for the worst case (lr_plan_bytes, several times
 * larger for wide supports) that also holds the build's transient arrays;
 * packing moves what the plan keeps into a buffer of this size, so that
 * many plans (one per chunk of a large data set) can stay resident.  0 for
 * a NULL plan. */
size_t lr_plan_packed_bytes(const lr_plan *plan);

/* Copy plan's arrays into buf (device, >= lr_plan_packed_bytes) on stream
 * and return a new handle over buf in *out, usable exactly as the original
 * (same results, bit for bit).  The original buffer may be reused or freed
 * once the copies have run on the stream; the original handle stays valid
 * while its buffer lives.  Release the new handle with lr_plan_free.
 * LR_E_WORKSPACE when buf is too small. */
lr_status lr_plan_pack(const lr_plan *plan, void *buf, size_t bytes, lr_stream stream,
                       lr_plan **out);

/* Number of groups, kept (row, channel) pairs and total pairs of a plan,
 * and the kernel taps its groups cover, sum over groups of S_k^2 (the
 * gridder and degridder each do one complex multiply-add per tap and
 * polarisation). */
lr_status lr_plan_info(const lr_plan *plan, int64_t *n_groups, int64_t *n_kept,
                       int64_t *n_pairs, int64_t *taps);

/* Deterministic order, process-wide (default off): with on != 0 every later
 * lr_grid, lr_grid_overwrite and lr_sumwt call forms its sums in an order
 * that does not depend on scheduling, so that repeated calls on the same
 * inputs (alone or beside other work on the device) give bit-identical
 * grids and sums of weights.  Group sums (the weighted sum of each group of
 * identical samples of the binning step) are stored, never added with
 * atomics: along tracks for groups one wavefront holds whole, otherwise
 * over fixed segments of the plan's sorted order, pieces joined in order;
 * sums of weights come from fixed per-(channel, row block) partials and
 * fixed trees; each grid tile is written by one workgroup, which takes the
 * tile's chunks in order, instead of atomic flushes of tiles shared by
 * several chunks.  Slower (about 2.2x per gridding call on data whose
 * samples merge into large groups); the results equal the default mode's
 * up to FP rounding order.  The workspace size of LR_OP_GRID and
 * LR_OP_SUMWT always includes what this mode needs.  lr_make_psf keeps its
 * atomic mirror adds.  Returns LR_OK.  lr_deterministic returns the current
 * setting (0 or 1). */
lr_status lr_set_deterministic(int32_t on);
int32_t lr_deterministic(void);

/* Diagnostic timing hook: the next lr_grid / lr_make_psf / lr_degrid on the
 * calling thread records `start` (a hipEvent_t) on its stream just before
 * its main kernel (the gridder or the degridder) and `stop` just after it,
 * then forgets both.  NULL, NULL clears a pending request. */
lr_status lr_set_profile_events(void *start, void *stop);

/* ---- the hot path ------------------------------------------------------------ */

/* Workspace of the visibility calls below (lr_grid, lr_grid_overwrite,
 * lr_degrid, lr_make_psf, lr_sumwt): `work` is device scratch of at least
 * lr_workspace_bytes(op, ...) bytes for the same arguments (the per-group
 * sums or values, and a transient plan when vis->plan is NULL); a smaller
 * work_bytes gives LR_E_WORKSPACE before anything is enqueued.  The
 * scratch is free again once the call's work has run on its stream. */

/* Gridding G (Eq. IMAGE-MOD): grid[P][pol][p_v + t_v][p_u + t_u] +=
 * Ct(o, t) phi(t) W V for every kept sample, Ct = C or conj C (w < 0),
 * phi = pointing phasor (Eq. CIJ) when ant ids and offsets are given.
 * With a Mueller table (pol_beam > 0) grid pol p receives sum_q Ct_qp
 * W_q V_q over the correlations q its column of the sparse matrix holds
 * (one gridder pass per kind; the time grows with the kinds).
 * sumwt [nplane][npol] (FP64) += W over kept samples; counters += class
 * counts.  sumwt and counters may be NULL. */
lr_status lr_grid(const lr_cf *cf, const lr_vis *vis, lr_precision precision, void *grid,
                  double *sumwt, int64_t *counters, void *work, size_t work_bytes,
                  lr_stream stream);

/* Gridding G as lr_grid, with the outputs replaced instead of accumulated:
 * grid = G(vis) (every cell of every plane and pol is written, cells no
 * footprint reaches become 0), sumwt = the sums of weights, counters = the
 * class counts.  The caller need not clear them first, so a fresh grid
 * costs one write pass instead of a clear plus a read-modify-write.
 * Arguments, layout, workspace and errors as lr_grid. */
lr_status lr_grid_overwrite(const lr_cf *cf, const lr_vis *vis, lr_precision precision,
                            void *grid, double *sumwt, int64_t *counters, void *work,
                            size_t work_bytes, lr_stream stream);

/* Gridding G as lr_grid (accumulating; same arguments, layout, results and
 * errors) for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * takes no workspace: the group sums (and the deterministic order's
 * partial sums) live in a fixed 64 MiB device array of the library, one
 * copy per GPU, held until the process ends; the call itself allocates
 * nothing.  vis->plan must be a built plan (LR_E_ARG otherwise).  Plans
 * whose scratch exceeds the array (more than 2,097,152 groups at 4 pols
 * in FP32, 1,048,576 in FP64, fewer in the deterministic order) give
 * LR_E_RANGE before anything is enqueued.  The array is shared by every
 * call on the same GPU: calls that overlap on one GPU (different streams
 * or threads) race and must be serialised by the caller.  The calling
 * thread's current device must be the device of `stream`. */
lr_status lr_grid_static(const lr_cf *cf, const lr_vis *vis, lr_precision precision,
                         void *grid, double *sumwt, int64_t *counters, lr_stream stream);

/* Degridding D (Eq. ME-MOD-GRIDDED): vis = sum_t conj(Ct(o, t) phi(t)) grid[...]
 * for kept samples; flagged and dropped samples are written as 0.  No
 * weights enter the sum.  counters may be NULL.  With a Mueller table
 * (pol_beam > 0) correlation q sums conj(Ct_qp) over the grid pols p its
 * row of the sparse matrix holds (one pass per kind).  The grid must hold
 * finite values: with FP32 grids the gather reads two cells per load and may
 * take in one cell beyond a footprint row's end with weight 0, so an Inf or
 * NaN there would reach the sample. */
lr_status lr_degrid(const lr_cf *cf, lr_vis *vis, lr_precision precision, const void *grid,
                    int64_t *counters, void *work, size_t work_bytes, lr_stream stream);

/* PSF: psf_grid += 1/2 (g + H g), g = the gridding of unit visibilities with
 * weights W under the PSF footprint rule, (H g)[i][j] = conj g[ny-i][nx-j].
 * The result is Hermitian, so its image is real.  vis->vis is not read.
 * Tables of one scalar beam only (LR_E_CF for pol_beam > 0). */
lr_status lr_make_psf(const lr_cf *cf, const lr_vis *vis, lr_precision precision,
                      void *psf_grid, double *sumwt, int64_t *counters, void *work,
                      size_t work_bytes, lr_stream stream);

/* Sum of weights per (plane, pol) in FP64 and class counts, under the
 * gridding footprint rule. */
lr_status lr_sumwt(const lr_cf *cf, const lr_vis *vis, lr_precision precision,
                   double *sumwt, int64_t *counters, void *work, size_t work_bytes,
                   lr_stream stream);

/* ---- image plane around the hot path (residual image, Eq. ResIm) ---------- */

/* Grid correction of plane (fg, k), which must be separable (PS only, or the
 * w = 0 plane of a PS + W table): C[o_v][o_u][t_v][t_u] = c1[o_v][t_v]
 * c1[o_u][t_u], with c1 the o_v = 0, t_v = 0 row over sqrt(C(0, 0)).  out
 * (device, complex128 [n]) = (1/O) sum over o in [-O/2, O/2) and t of
 * c1[o][t] exp(2 pi i (t - o/O) xi), xi = (i - n/2)/n: the mean image-plane
 * response of one sample.  LR_E_ARG for a plane with an A or W (k > 0)
 * term, LR_E_RANGE for (fg, k) outside the table. */
lr_status lr_gcf(const lr_cf *cf, int32_t fg, int32_t k, int32_t n, void *out,
                 lr_stream stream);

/* out[P][pol][iy][ix] = Re(img[P][pol][iy][ix]) / (gcf_x[ix] gcf_y[iy]
 * sumwt[P][pol]): the normalisation of F^dagger(grid) (computed by the
 * caller, e.g. with rocFFT) into an image.  img is complex128 (LR_F64) or
 * complex64 (other forms), out float64 or float32 of the grid's shape;
 * gcf_x [nx], gcf_y [ny], sumwt [nplane][npol] are FP64; all device. */
lr_status lr_image_normalize(const lr_cf *cf, lr_precision precision, const void *img,
                             const double *gcf_x, const double *gcf_y, const double *sumwt,
                             void *out, lr_stream stream);

/* The grid correction of tables whose planes are not separable (an A term,
 * or W planes beyond w = 0; Table AWP-CFSETUP): the PS term's taper that
 * the kernels carry, at n image pixels, out[i] = psi_0(c, 2 (i - n/2) / n),
 * c = pi S_ps / 2 (1 without a PS term).  out: device float64 [n]. */
lr_status lr_ps_taper(const lr_cf *cf, int32_t n, void *out, lr_stream stream);

/* Weight image of A-projection (the normalisation of Eq. ResIm's image when
 * the kernels of G carry the A term; Table AWP-CFSETUP A-Projection rows):
 * the data hold the beam once and G applies it again, so a source at (l, m)
 * images with
 *     out[P][pol][iy][ix] = sum_fg w[P][pol][fg] B_fg(rho)^2 / sum_fg w[P][pol][fg],
 * B_fg = the table's A term (Airy power pattern of the dish at the group's
 * frequency), rho = sqrt(l^2 + m^2), (l, m) = ((ix - nx/2) cell_l,
 * (iy - ny/2) cell_m); 1 everywhere without an A term, 0 where the weights
 * sum to 0.  fg_weight: device float64 [nplane][npol][n_fg], the sums of
 * weights of each frequency group's channels (lr_sumwt on those channels);
 * out: device float64 [nplane][npol][ny][nx].  Tables of a scalar beam only
 * (LR_E_CF for pol_beam > 0: a polarised beam mixes the pols). */
lr_status lr_pb_image(const lr_cf *cf, const double *fg_weight, void *out, lr_stream stream);

/* lr_image_normalize with the weight image: out = Re(img) / (gcf_x[ix]
 * gcf_y[iy] sumwt[P][pol] pb[P][pol][iy][ix]) where pb >= pb_min, 0 where
 * it is below (outside the usable beam).  pb: device float64 of the image's
 * shape (lr_pb_image); gcf_x, gcf_y typically from lr_ps_taper.  LR_E_ARG
 * for pb_min <= 0. */
lr_status lr_image_normalize_pb(const lr_cf *cf, lr_precision precision, const void *img,
                                const double *gcf_x, const double *gcf_y, const double *sumwt,
                                const double *pb, double pb_min, void *out, lr_stream stream);

/* ---- mosaic rows of the imaging-mode table (Eq. CIJ) --------------------- */

/* Change of phase centre of mosaic data, in place: every sample of a row
 * whose field f is in [0, nfield) is multiplied by
 *     exp(sign 2 pi i (u l_f + v m_f)),  u = u_m nu / c, v = v_m nu / c,
 * the argument formed in FP64 and reduced modulo 1; sign = -1 for
 * direction < 0 (from the field's phase centre s(P) to the joint image
 * centre s0, before gridding), +1 otherwise (back, after degridding).  The
 * w-term of the change is not applied (flat-sky shift).  The kernel shift
 * of a field is the pointing phasor of lr_grid / lr_degrid on virtual
 * antennas f * nant + a with offsets ant_dlm[a] + field_dlm[f].
 *   vis        [nrow][nchan][npol] complex128 (LR_F64) or complex64 (LR_F32),
 *              device, updated in place
 *   uvw        [nrow][3] metres, device;  freq_hz [nchan] host
 *   field      [nrow] int32, device (rows outside [0, nfield) unchanged)
 *   field_dlm  [nfield][2] (l, m) of each field's phase centre relative to
 *              the image centre, direction cosines, device
 * LR_E_ARG for NULL pointers or negative sizes, LR_E_DTYPE for other
 * precisions. */
lr_status lr_rephase(int64_t nrow, int32_t nchan, int32_t npol, lr_precision precision,
                     void *vis, const double *uvw, const double *freq_hz, const int32_t *field,
                     const double *field_dlm, int32_t nfield, int32_t direction,
                     lr_stream stream);

/* ---- calibration: diagonal G-Jones (the calibration section) -------------- */

/* PreSolvePrep (Eq. VAvg): ratio averages of observed to model visibilities
 * per solution interval, parallel hand and baseline, as inputs of the gain
 * solve.  For every kept sample (weight > 0, model != 0, ant1 != ant2, row
 * and channel inside an interval) of baseline (i, j):
 *     X[s][q][i][j] = sum W V conj(M) / sum W |M|^2,
 *     w[s][q][i][j] = sum W |M|^2,
 * the inverse-variance mean of the ratios V / M, so that X estimates
 * g_i conj(g_j) (the paper's sum of ratios normalised by its weights).
 * X[s][q][j][i] = conj(X[s][q][i][j]); rows j-i and i-j enter the same
 * average; the diagonal and baselines without samples are 0.
 *   vis_obs, vis_model  [nrow][nchan][npol] complex (complex128 with
 *                       LR_F64, complex64 with LR_F32), device
 *   weight              [nrow][nchan][npol] float64 / float32, device; NULL
 *                       for unit weights
 *   ant1, ant2          [nrow] int32 antenna ids, device; ids outside
 *                       [0, nant) are ignored
 *   row_sol [nrow], chan_sol [nchan]  int32 interval of each row / channel,
 *                       device; < 0 or >= n_tsol / n_fsol: not used
 *   rows_per_step       rows of one dump of time-major data (the number of
 *                       baselines), or 1: only the speed depends on it
 *   X                   complex128 [n_tsol][n_fsol][npar][nant][nant],
 *   w                   float64 of the same shape, device, overwritten;
 *                       s = t_sol * n_fsol + f_sol; npar = 2 parallel hands
 *                       (XX, YY of 4 correlations; both of 2), 1 for npol 1
 * Sums in FP64.  LR_E_ARG for NULL pointers or sizes out of range,
 * LR_E_DTYPE for a precision other than LR_F64 / LR_F32. */
lr_status lr_cal_vavg(int64_t nrow, int32_t nchan, int32_t npol, lr_precision precision,
                      const void *vis_obs, const void *vis_model, const void *weight,
                      const int32_t *ant1, const int32_t *ant2, int32_t nant,
                      const int32_t *row_sol, int32_t n_tsol, const int32_t *chan_sol,
                      int32_t n_fsol, int32_t rows_per_step, double *X, double *w,
                      lr_stream stream);

/* UpdateDir, ModelUpdate and ExitCriteria (Eqs. CalUpdateDir,
 * CalUpdateModel): for each of n_problems independent problems (X, w of
 * lr_cal_vavg, consecutive [nant][nant] matrices) iterate, from the gains
 * in g (complex128 [n_problems][nant], device, in / out),
 *     dg_i = sum_{j != i} g_j X_ij w_ij / sum_{j != i} |g_j|^2 w_ij
 *     g_i <- (1 - alpha) g_i + alpha dg_i      (all i from the same iterate;
 *                                              no weight: g_i unchanged)
 * until max_i |change| < delta or max_iter iterations.  iterations
 * (int32 [n_problems]) and change (float64 [n_problems]: the last max
 * |change|) receive the outcome, device.  FP64.  LR_E_ARG for NULL
 * pointers, nant outside [1, 2048], alpha outside (0, 1], delta < 0 or
 * max_iter < 0. */
lr_status lr_cal_solve(const double *X, const double *w, int32_t nant, int64_t n_problems,
                       double alpha, double delta, int32_t max_iter, double *g,
                       int32_t *iterations, double *change, lr_stream stream);

/* ---- minor cycle (ModelUpdate of the imaging section) -------------------- */

/* Hogbom minor cycle on one image plane [ny][nx] (float64 with LR_F64,
 * float32 with LR_F32; all device): repeatedly take the pixel of largest
 * |residual| (lowest row-major index on ties); stop when it is below
 * `threshold` or `niter` subtractions are done; otherwise add gain x peak
 * to model at that pixel and subtract gain x peak x psf from the
 * overlapping part of residual, with the psf's centre (ny/2, nx/2) on the
 * peak.  residual is updated in place, model accumulated.  *iterations
 * (host) receives the number of subtractions; the call synchronises the
 * stream to read it.  work: device scratch of lr_hogbom_work_bytes bytes.
 * LR_E_ARG for gain outside (0, 1] or niter < 0. */
size_t lr_hogbom_work_bytes(int32_t nx, int32_t ny);
lr_status lr_hogbom(const void *psf, void *residual, void *model, int32_t nx, int32_t ny,
                    lr_precision precision, double gain, double threshold, int32_t niter,
                    int32_t *iterations, void *work, size_t work_bytes, lr_stream stream);

/* Test hook: the index map of every (row, channel) as int32
 * out[nrow][nchan][8] = {p_u, p_v, o_u, o_v, k, conj, keep, fg} (device). */
lr_status lr_debug_map(const lr_cf *cf, const lr_vis *vis, int psf, int32_t *out,
                       lr_stream stream);

const char *lr_status_str(lr_status s);
const char *lr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LR_H */
