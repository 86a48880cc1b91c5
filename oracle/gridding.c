/*
 * CPU FP64 oracle for convolutional gridding and degridding.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and
 * the benchmark's CPU-baseline leg load it.  It shares no code with the GPU
 * library and must never be called from the product path.
 *
 * What it computes (paper: Eq. ME-MOD-GRIDDED for degridding D, Eq. IMAGE-MOD
 * for gridding G with the weights inside the sum, Eq. ResIm for the use of
 * G on weighted residuals, Eq. CIJ for the per-baseline pointing phasor):
 *
 *   map      (row, chan) -> pixel p, oversampling offset o, w-plane k, conj flag
 *   grid     grid[P][pol][p_v + t_v][p_u + t_u] += Ct(o, t) * phi(t) * W * V
 *   degrid   V = sum_t conj(Ct(o, t) * phi(t)) * grid[P][pol][p_v + t_v][p_u + t_u]
 *
 * With a sparse Mueller matrix of CFs (the table holds several kinds, and
 * mueller[q * npol + p] is the kind of element M[q][p], -1 for none), the
 * pols mix: grid pol p receives sum_q Ct_qp W_q V_q, and V_q = sum_p
 * conj(Ct_qp) grid_p.  Without one, M is the identity times the one table.
 *   sumwt    sum of W over kept samples, per (plane, pol)
 *   psf      1/2 (g + H g), g = unit-visibility weight grid, (H g)[i][j] =
 *            conj g[ny - i][nx - j]
 *
 * Ct = C (w >= 0) or conj C (w < 0, when there is more than one w-plane).
 * All arithmetic is FP64, samples are visited in input order, taps in
 * (t_v, t_u) row-major order.  Complex numbers are interleaved (re, im).
 *
 * Compile with -O2 -ffp-contract=off: the index map relies on exactly one
 * rounding in fma() and no other contraction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, ny, npol, nplane;
    int32_t O, n_w, n_fg, psf;        /* psf != 0: footprint must stay in [1, N-1] */
    const int32_t *h;                 /* [n_w] half-widths */
    const int64_t *plane_off;         /* [n_fg * n_w] complex offset of plane (fg, k) */
    const double *cf;                 /* interleaved complex table */
    int64_t nrow;
    int32_t nchan;
    const double *uvw;                /* [nrow][3] metres */
    const double *kx, *ky, *kw;       /* [nchan] per-channel scale constants */
    double ox, oy;
    const int32_t *chan_plane;        /* [nchan], < 0 = skip */
    const int32_t *chan_fg;           /* [nchan] */
    /* pointing-offset phasor (Eq. CIJ); ant1 == NULL disables it */
    const int32_t *ant1, *ant2;       /* [nrow] */
    const double *ant_dlm;            /* [nant][2] radians */
    const double *f_scale;            /* [nchan]: pi * D * nu / c */
    double du_dl, dv_dm;              /* uv cell size times... see phasor() */
    const int32_t *mueller;           /* [npol][npol] kind of M[q][p], -1 none; NULL: diagonal */
    int64_t kind_stride;              /* complex elements per kind */
} octx;

typedef struct {
    int32_t pu, pv, ou, ov, k, conj, keep, fg;
} omap;

/* floor division for a positive divisor */
static int64_t floordiv(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b) != 0 && ((a < 0) != (b < 0))) q -= 1;
    return q;
}

/* Index map of one (row, chan): Eq. IMAGE-MOD places the visibility at its
 * (u, v) on the regular grid; the reading used here rounds the position in
 * units of 1/O cell half-up, splits it into pixel p and offset o in
 * [-O/2, O/2), and picks the w-plane by rounding |w| on a linear scale. */
static omap map_one(const octx *c, int64_t r, int32_t ch) {
    omap m;
    memset(&m, 0, sizeof m);
    double u = c->uvw[3 * r + 0], v = c->uvw[3 * r + 1], w = c->uvw[3 * r + 2];
    m.fg = c->chan_fg ? c->chan_fg[ch] : 0;
    double X = fma(u, c->kx[ch], c->ox);
    double Y = fma(v, c->ky[ch], c->oy);
    double limx = (double)c->nx * (double)c->O;
    double limy = (double)c->ny * (double)c->O;
    if (!(X >= 0.0 && X < limx) || !(Y >= 0.0 && Y < limy)) return m;
    int64_t qx = (int64_t)floor(X);
    int64_t qy = (int64_t)floor(Y);
    int64_t half = c->O / 2;
    int64_t px = floordiv(qx + half, c->O);
    int64_t py = floordiv(qy + half, c->O);
    m.pu = (int32_t)px;
    m.pv = (int32_t)py;
    m.ou = (int32_t)(qx - px * c->O);
    m.ov = (int32_t)(qy - py * c->O);
    double kk = floor(fma(fabs(w), c->kw[ch], 0.5));
    if (!(kk <= (double)(c->n_w - 1))) return m;
    m.k = (int32_t)kk;
    m.conj = (c->n_w > 1 && w < 0.0) ? 1 : 0;
    int32_t h = c->h[m.k];
    int32_t lo = c->psf ? 1 : 0;
    if (m.pu - h < lo || m.pu + h > c->nx - 1) return m;
    if (m.pv - h < lo || m.pv + h > c->ny - 1) return m;
    m.keep = 1;
    return m;
}

/* Per-sample pointing phasor, Eq. CIJ read as a shift of the beam by the
 * baseline-mean offset ds = (ds_1 + ds_2)/2 times the loss factor
 * f(ds_1 - ds_2) = [2 J1(x)/x]^2 at x = pi D nu |ds_1 - ds_2| / (2c).
 * phi(t) = f * exp(-2 pi i (t_u - o_u/O) du dl) * exp(-2 pi i (t_v - o_v/O) dv dm);
 * each argument is formed in FP64 as (t O - o) * (du dl / O) and reduced
 * modulo 1 before the sine and cosine. */
static void phasor_1d(int32_t h, int32_t O, int32_t o, double beta, double *re, double *im) {
    for (int32_t t = -h; t <= h; ++t) {
        double a = (double)(t * O - o) * beta;
        a = a - nearbyint(a);
        double ph = -2.0 * M_PI * a;
        re[t + h] = cos(ph);
        im[t + h] = sin(ph);
    }
}

static double airy_power(double x) {
    if (x == 0.0) return 1.0;
    double j = jn(1, x);
    double b = 2.0 * j / x;
    return b * b;
}

/* 0 if no phasor; else fills f, phu, phv (length 2h+1 each) */
static int phasor(const octx *c, int64_t r, int32_t ch, const omap *m, double *f,
                  double *phur, double *phui, double *phvr, double *phvi) {
    if (!c->ant1) return 0;
    int32_t a1 = c->ant1[r], a2 = c->ant2[r];
    double l1 = c->ant_dlm[2 * a1], m1 = c->ant_dlm[2 * a1 + 1];
    double l2 = c->ant_dlm[2 * a2], m2 = c->ant_dlm[2 * a2 + 1];
    double dl = 0.5 * (l1 + l2), dm = 0.5 * (m1 + m2);
    double ddl = l1 - l2, ddm = m1 - m2;
    double dist = sqrt(ddl * ddl + ddm * ddm);
    *f = airy_power(c->f_scale[ch] * 0.5 * dist);
    int32_t h = c->h[m->k];
    phasor_1d(h, c->O, m->ou, (c->du_dl * dl) / (double)c->O, phur, phui);
    phasor_1d(h, c->O, m->ov, (c->dv_dm * dm) / (double)c->O, phvr, phvi);
    return 1;
}

/* Pointer to table entry C[kind][fg][k][ov + O/2][ou + O/2][0][0] */
static const double *cf_sub(const octx *c, const omap *m, int32_t kind) {
    int32_t S = 2 * c->h[m->k] + 1;
    int64_t no = c->O + 1;
    int64_t idx = (int64_t)kind * c->kind_stride +
                  c->plane_off[(int64_t)m->fg * c->n_w + m->k] +
                  (((int64_t)(m->ov + c->O / 2) * no + (m->ou + c->O / 2)) * S * S);
    return c->cf + 2 * idx;
}

/* Kind of Mueller element M[q][p] (-1: none) */
static int32_t kind_of(const octx *c, int32_t q, int32_t p) {
    if (c->mueller) return c->mueller[q * c->npol + p];
    return q == p ? 0 : -1;
}

void oracle_map(const octx *c, int32_t *out) {
    for (int64_t r = 0; r < c->nrow; ++r)
        for (int32_t ch = 0; ch < c->nchan; ++ch) {
            omap m = map_one(c, r, ch);
            int32_t *o = out + 8 * (r * c->nchan + ch);
            o[0] = m.pu; o[1] = m.pv; o[2] = m.ou; o[3] = m.ov;
            o[4] = m.k; o[5] = m.conj; o[6] = m.keep; o[7] = m.fg;
        }
}

/* counters[0] kept, [1] flagged, [2] dropped; sumwt[plane][pol] */
void oracle_sumwt(const octx *c, const double *weight, double *sumwt, int64_t *counters) {
    for (int64_t r = 0; r < c->nrow; ++r)
        for (int32_t ch = 0; ch < c->nchan; ++ch) {
            int32_t P = c->chan_plane[ch];
            omap m;
            if (P >= 0) m = map_one(c, r, ch);
            for (int32_t p = 0; p < c->npol; ++p) {
                double W = weight[(r * c->nchan + ch) * c->npol + p];
                if (P < 0 || W == 0.0) { counters[1]++; continue; }
                if (!m.keep) { counters[2]++; continue; }
                counters[0]++;
                sumwt[P * c->npol + p] += W;
            }
        }
}

/* Gridding, parallel over disjoint strips of grid rows; every thread visits
 * all samples in input order, so each cell sees the serial order of adds. */
void oracle_grid(const octx *c, const double *vis, const double *weight, double *grid,
                 int unit_vis, int nthreads) {
    const int64_t plane = (int64_t)c->nx * c->ny;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
#endif
    {
        int tid = 0, nt = 1;
#ifdef _OPENMP
        tid = omp_get_thread_num();
        nt = omp_get_num_threads();
#endif
        int32_t y0 = (int32_t)(((int64_t)c->ny * tid) / nt);
        int32_t y1 = (int32_t)(((int64_t)c->ny * (tid + 1)) / nt);
        int32_t hmax = 0;
        for (int i = 0; i < c->n_w; ++i) if (c->h[i] > hmax) hmax = c->h[i];
        double *phur = malloc(sizeof(double) * (2 * hmax + 1) * 4);
        double *phui = phur + (2 * hmax + 1), *phvr = phui + (2 * hmax + 1),
               *phvi = phvr + (2 * hmax + 1);
        for (int64_t r = 0; r < c->nrow; ++r)
            for (int32_t ch = 0; ch < c->nchan; ++ch) {
                int32_t P = c->chan_plane[ch];
                if (P < 0) continue;
                omap m = map_one(c, r, ch);
                if (!m.keep) continue;
                int32_t h = c->h[m.k], S = 2 * h + 1;
                if (m.pv + h < y0 || m.pv - h >= y1) continue;
                double f = 1.0;
                int po = phasor(c, r, ch, &m, &f, phur, phui, phvr, phvi);
                double csign = m.conj ? -1.0 : 1.0;
                for (int32_t p = 0; p < c->npol; ++p)
                for (int32_t q = 0; q < c->npol; ++q) {
                    int32_t kind = kind_of(c, q, p);
                    if (kind < 0) continue;
                    const double *C = cf_sub(c, &m, kind);
                    int64_t s = (r * c->nchan + ch) * c->npol + q;
                    double W = weight[s];
                    if (W == 0.0) continue;
                    double ar, ai;
                    if (unit_vis) { ar = W; ai = 0.0; }
                    else { ar = W * vis[2 * s]; ai = W * vis[2 * s + 1]; }
                    double *g = grid + 2 * (((int64_t)P * c->npol + p) * plane);
                    for (int32_t tv = -h; tv <= h; ++tv) {
                        int32_t y = m.pv + tv;
                        if (y < y0 || y >= y1) continue;
                        for (int32_t tu = -h; tu <= h; ++tu) {
                            int64_t ti = (int64_t)(tv + h) * S + (tu + h);
                            double cr = C[2 * ti], ci = csign * C[2 * ti + 1];
                            if (po) {
                                double pr = phur[tu + h] * phvr[tv + h] - phui[tu + h] * phvi[tv + h];
                                double pi = phur[tu + h] * phvi[tv + h] + phui[tu + h] * phvr[tv + h];
                                pr *= f; pi *= f;
                                double nr = cr * pr - ci * pi, ni = cr * pi + ci * pr;
                                cr = nr; ci = ni;
                            }
                            int64_t gi = (int64_t)y * c->nx + (m.pu + tu);
                            g[2 * gi] += cr * ar - ci * ai;
                            g[2 * gi + 1] += cr * ai + ci * ar;
                        }
                    }
                }
            }
        free(phur);
    }
}

/* Degridding: V = sum_t conj(Ct * phi) * grid; flagged (weight == 0, when a
 * weight array is given), skipped-channel and dropped samples are set to 0. */
void oracle_degrid(const octx *c, const double *grid, const double *weight, double *vis,
                   int nthreads) {
    const int64_t plane = (int64_t)c->nx * c->ny;
    int32_t hmax = 0;
    for (int i = 0; i < c->n_w; ++i) if (c->h[i] > hmax) hmax = c->h[i];
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
#endif
    {
        double *phur = malloc(sizeof(double) * (2 * hmax + 1) * 4);
        double *phui = phur + (2 * hmax + 1), *phvr = phui + (2 * hmax + 1),
               *phvi = phvr + (2 * hmax + 1);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t r = 0; r < c->nrow; ++r)
            for (int32_t ch = 0; ch < c->nchan; ++ch) {
                int32_t P = c->chan_plane[ch];
                omap m;
                memset(&m, 0, sizeof m);
                if (P >= 0) m = map_one(c, r, ch);
                double f = 1.0;
                int po = 0;
                if (m.keep) po = phasor(c, r, ch, &m, &f, phur, phui, phvr, phvi);
                for (int32_t q = 0; q < c->npol; ++q) {
                    int64_t s = (r * c->nchan + ch) * c->npol + q;
                    vis[2 * s] = 0.0;
                    vis[2 * s + 1] = 0.0;
                    if (!m.keep) continue;
                    if (weight && weight[s] == 0.0) continue;
                    int32_t h = c->h[m.k], S = 2 * h + 1;
                    double csign = m.conj ? -1.0 : 1.0;
                    double sr = 0.0, si = 0.0;
                    for (int32_t p = 0; p < c->npol; ++p) {
                    int32_t kind = kind_of(c, q, p);
                    if (kind < 0) continue;
                    const double *C = cf_sub(c, &m, kind);
                    const double *g = grid + 2 * (((int64_t)P * c->npol + p) * plane);
                    for (int32_t tv = -h; tv <= h; ++tv)
                        for (int32_t tu = -h; tu <= h; ++tu) {
                            int64_t ti = (int64_t)(tv + h) * S + (tu + h);
                            double cr = C[2 * ti], ci = csign * C[2 * ti + 1];
                            if (po) {
                                double pr = phur[tu + h] * phvr[tv + h] - phui[tu + h] * phvi[tv + h];
                                double pi = phur[tu + h] * phvi[tv + h] + phui[tu + h] * phvr[tv + h];
                                pr *= f; pi *= f;
                                double nr = cr * pr - ci * pi, ni = cr * pi + ci * pr;
                                cr = nr; ci = ni;
                            }
                            int64_t gi = (int64_t)(m.pv + tv) * c->nx + (m.pu + tu);
                            double gr = g[2 * gi], gim = g[2 * gi + 1];
                            /* conj(c) * g */
                            sr += cr * gr + ci * gim;
                            si += cr * gim - ci * gr;
                        }
                    }
                    vis[2 * s] = sr;
                    vis[2 * s + 1] = si;
                }
            }
        free(phur);
    }
}

/* Hermitian symmetrisation: out = 1/2 (g + H g), H g[i][j] = conj g[ny-i][nx-j];
 * row/column 0 have no mirror inside the grid and are taken as 1/2 g. */
void oracle_hermitian_sym(const octx *c, const double *g, double *out) {
    const int64_t nx = c->nx, ny = c->ny;
    for (int64_t pl = 0; pl < (int64_t)c->nplane * c->npol; ++pl) {
        const double *a = g + 2 * pl * nx * ny;
        double *b = out + 2 * pl * nx * ny;
        for (int64_t i = 0; i < ny; ++i)
            for (int64_t j = 0; j < nx; ++j) {
                double re = a[2 * (i * nx + j)], im = a[2 * (i * nx + j) + 1];
                double mr = 0.0, mi = 0.0;
                if (i > 0 && j > 0) {
                    int64_t mm = (ny - i) * nx + (nx - j);
                    mr = a[2 * mm];
                    mi = -a[2 * mm + 1];
                }
                b[2 * (i * nx + j)] = 0.5 * (re + mr);
                b[2 * (i * nx + j) + 1] = 0.5 * (im + mi);
            }
    }
}

/* PSF by mirror scatter, the alternative construction: each kept sample adds
 * 1/2 W Ct(o,t) phi(t) at p + t and 1/2 conj(W Ct(o,t) phi(t)) at N - p - t.
 * Serial; used only as a cross-check of the symmetrisation pass. */
void oracle_psf_mirror(const octx *c, const double *weight, double *grid) {
    const int64_t plane = (int64_t)c->nx * c->ny;
    int32_t hmax = 0;
    for (int i = 0; i < c->n_w; ++i) if (c->h[i] > hmax) hmax = c->h[i];
    double *phur = malloc(sizeof(double) * (2 * hmax + 1) * 4);
    double *phui = phur + (2 * hmax + 1), *phvr = phui + (2 * hmax + 1),
           *phvi = phvr + (2 * hmax + 1);
    for (int64_t r = 0; r < c->nrow; ++r)
        for (int32_t ch = 0; ch < c->nchan; ++ch) {
            int32_t P = c->chan_plane[ch];
            if (P < 0) continue;
            omap m = map_one(c, r, ch);
            if (!m.keep) continue;
            int32_t h = c->h[m.k], S = 2 * h + 1;
            double f = 1.0;
            int po = phasor(c, r, ch, &m, &f, phur, phui, phvr, phvi);
            const double *C = cf_sub(c, &m, 0);
            double csign = m.conj ? -1.0 : 1.0;
            for (int32_t p = 0; p < c->npol; ++p) {
                int64_t s = (r * c->nchan + ch) * c->npol + p;
                double W = weight[s];
                if (W == 0.0) continue;
                double *g = grid + 2 * (((int64_t)P * c->npol + p) * plane);
                for (int32_t tv = -h; tv <= h; ++tv)
                    for (int32_t tu = -h; tu <= h; ++tu) {
                        int64_t ti = (int64_t)(tv + h) * S + (tu + h);
                        double cr = C[2 * ti], ci = csign * C[2 * ti + 1];
                        if (po) {
                            double pr = phur[tu + h] * phvr[tv + h] - phui[tu + h] * phvi[tv + h];
                            double pi = phur[tu + h] * phvi[tv + h] + phui[tu + h] * phvr[tv + h];
                            pr *= f; pi *= f;
                            double nr = cr * pr - ci * pi, ni = cr * pi + ci * pr;
                            cr = nr; ci = ni;
                        }
                        double vr = 0.5 * W * cr, vi = 0.5 * W * ci;
                        int64_t gi = (int64_t)(m.pv + tv) * c->nx + (m.pu + tu);
                        int64_t mi = (int64_t)(c->ny - m.pv - tv) * c->nx + (c->nx - m.pu - tu);
                        g[2 * gi] += vr;
                        g[2 * gi + 1] += vi;
                        g[2 * mi] += vr;
                        g[2 * mi + 1] -= vi;
                    }
            }
        }
    free(phur);
}
