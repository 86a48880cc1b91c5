// C ABI of the gfx950 gridding library: validation, derived geometry,
// workspace carving and dispatch to the kernels.  All host arithmetic that
// feeds the bit-exact index map is FP64 without contraction (this file is
// compiled with -ffp-contract=off).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "lr_internal.h"
#include "lr_launch.h"

using namespace lr;

namespace {

thread_local std::string g_err;
thread_local hipEvent_t g_prof_start = nullptr, g_prof_stop = nullptr;
// deterministic gridding sums (lr_set_deterministic), process-wide
std::atomic<int> g_det{0};

// Record the pending profile events around the main kernel of a call.
struct ProfileScope {
    hipStream_t s;
    hipEvent_t a, b;
    explicit ProfileScope(hipStream_t st) : s(st), a(g_prof_start), b(g_prof_stop) {
        g_prof_start = g_prof_stop = nullptr;
    }
    void begin() { if (a) (void)hipEventRecord(a, s); }
    void end() { if (b) (void)hipEventRecord(b, s); }
};

lr_status fail(lr_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

lr_status dev_fail(hipError_t e, const char *what) {
    return fail(LR_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int bitwidth(int64_t maxval) {
    int b = 0;
    while (maxval > 0) { ++b; maxval >>= 1; }
    return b;
}

std::vector<int32_t> half_widths(int32_t n_w, int32_t h_min, int32_t h_max) {
    std::vector<int32_t> h(n_w);
    if (n_w == 1) { h[0] = h_min; return h; }
    for (int64_t k = 0; k < n_w; ++k)
        h[k] = (int32_t)(h_min + (2 * (int64_t)(h_max - h_min) * k + n_w - 1) / (2 * (int64_t)(n_w - 1)));
    return h;
}

size_t elem_bytes_of(lr_precision p) {
    switch (p) {
        case LR_F64: return 16;
        case LR_F32: return 8;
        case LR_F32_CF16:
        case LR_F32_CFBF16: return 4;
    }
    return 0;
}

lr_status check_grid(const lr_grid_spec *g) {
    if (!g) return fail(LR_E_ARG, "grid spec is NULL");
    if (g->nx < 8 || g->ny < 8 || (g->nx & 1) || (g->ny & 1))
        return fail(LR_E_ARG, "nx, ny must be even and >= 8 (got %d x %d)", g->nx, g->ny);
    if (g->nx > 16384 || g->ny > 16384) return fail(LR_E_RANGE, "nx, ny must be <= 16384");
    if (!(g->npol == 1 || g->npol == 2 || g->npol == 4))
        return fail(LR_E_ARG, "npol must be 1, 2 or 4 (got %d)", g->npol);
    if (g->nplane < 1 || g->nplane > 4096) return fail(LR_E_ARG, "nplane must be in 1..4096");
    if (!(g->cell_l > 0.0) || !(g->cell_m > 0.0) || !std::isfinite(g->cell_l) ||
        !std::isfinite(g->cell_m))
        return fail(LR_E_ARG, "cell sizes must be positive and finite");
    return LR_OK;
}

lr_status check_spec(const lr_cf_spec *s) {
    if (!s) return fail(LR_E_ARG, "cf spec is NULL");
    if (s->terms == 0 || (s->terms & ~7u)) return fail(LR_E_ARG, "terms must be a nonzero set of PS|W|A");
    if (s->oversample < 2 || s->oversample > 126 || (s->oversample & 1))
        return fail(LR_E_ARG, "oversample must be even in 2..126 (got %d)", s->oversample);
    if (s->n_w < 1 || s->n_w > 255) return fail(LR_E_ARG, "n_w must be in 1..255");
    if (s->n_w > 1 && !(s->w_max > 0.0 && std::isfinite(s->w_max)))
        return fail(LR_E_ARG, "w_max must be positive when n_w > 1");
    if (s->h_min < 0 || s->h_max < s->h_min || s->h_max > 128)
        return fail(LR_E_ARG, "need 0 <= h_min <= h_max <= 128");
    if (s->n_w == 1 && s->h_min != s->h_max)
        return fail(LR_E_ARG, "a single w-plane needs h_min == h_max");
    if (s->n_fg < 1 || s->n_fg > 127) return fail(LR_E_ARG, "n_fg must be in 1..127");
    if (!s->fg_hz) return fail(LR_E_ARG, "fg_hz is NULL");
    for (int i = 0; i < s->n_fg; ++i)
        if (!(s->fg_hz[i] > 0.0) || !std::isfinite(s->fg_hz[i]))
            return fail(LR_E_ARG, "fg_hz[%d] must be positive", i);
    if ((s->terms & LR_TERM_PS) && (s->ps_support < 1 || s->ps_support > 64))
        return fail(LR_E_ARG, "ps_support must be in 1..64");
    if ((s->terms & LR_TERM_A) && !(s->dish_m > 0.0)) return fail(LR_E_ARG, "dish_m must be positive");
    if (s->screen_m < 0 || (s->screen_m & 1)) return fail(LR_E_ARG, "screen_m must be even (0 = auto)");
    if (elem_bytes_of(s->storage) == 0) return fail(LR_E_DTYPE, "unknown storage type");
    if (s->pol_beam < 0 || s->pol_beam > 3) return fail(LR_E_ARG, "pol_beam must be in 0..3");
    if (s->pol_beam) {
        if (!(s->terms & LR_TERM_A)) return fail(LR_E_ARG, "a polarised beam needs the A term");
        if (!(std::fabs(s->beam_ellipticity) < 0.5))
            return fail(LR_E_ARG, "beam_ellipticity must lie in (-0.5, 0.5)");
        if (!(std::fabs(s->beam_leakage) <= 10.0))
            return fail(LR_E_ARG, "beam_leakage must lie in [-10, 10]");
    }
    return LR_OK;
}

// Mueller kinds of the polarised beam: element M[q][p] = J[q1][p1] J[q2][p2]
// of J = [[E_X, d], [d, E_Y]] (q = 2 q1 + q2) is the product of two of
// E_X, E_Y, d; its order is the number of d factors.  Kinds in table order:
// E_X^2, E_Y^2, E_X E_Y, E_X d, E_Y d, d^2.  Elements of order >= pol_beam
// are left out (-1).  The scalar beam has one kind on the diagonal.
int32_t n_kind_of(int32_t pol_beam) {
    static const int32_t n[4] = {1, 3, 5, 6};
    return n[pol_beam];
}

void kind_map(int32_t pol_beam, int32_t npol, int32_t out[16]) {
    for (int i = 0; i < 16; ++i) out[i] = -1;
    if (!pol_beam) {
        for (int q = 0; q < npol; ++q) out[q * 4 + q] = 0;
        return;
    }
    enum { EX = 0, EY = 1, D = 2 };
    auto el = [](int a, int b) { return a != b ? D : (a == 0 ? EX : EY); };
    for (int q = 0; q < 4; ++q)
        for (int p = 0; p < 4; ++p) {
            int f1 = el(q >> 1, p >> 1), f2 = el(q & 1, p & 1);
            int order = (f1 == D) + (f2 == D);
            if (order >= pol_beam) continue;
            if (f1 > f2) std::swap(f1, f2);
            int kind;
            if (f1 == EX && f2 == EX) kind = 0;
            else if (f1 == EY && f2 == EY) kind = 1;
            else if (f1 == EX && f2 == EY) kind = 2;
            else if (f1 == EX && f2 == D) kind = 3;
            else if (f1 == EY && f2 == D) kind = 4;
            else kind = 5;
            out[q * 4 + p] = kind;
        }
}

// The mask of one Mueller pass: bit q * npol + p when M[q][p] has `kind`.
uint32_t kind_mask(const lr_cf *cf, int32_t kind, int32_t npol) {
    uint32_t m = 0;
    for (int q = 0; q < npol; ++q)
        for (int p = 0; p < npol; ++p)
            if (cf->kind_of[q * 4 + p] == kind) m |= 1u << (q * npol + p);
    return m;
}

constexpr size_t kTablePad = 256;

struct Geometry {
    std::vector<int32_t> h;
    int32_t M = 0, hmax = 0;
    std::vector<int64_t> plane_off;
    int64_t n_elems = 0;            // per kind
    int32_t n_kind = 1;
    size_t off_h = 0, off_po = 0, off_exp = 0, off_scale = 0, off_table = 0, total = 0;
};

lr_status geometry(const lr_cf_spec *s, const lr_grid_spec *g, Geometry &G) {
    lr_status st;
    if ((st = check_spec(s)) != LR_OK) return st;
    if ((st = check_grid(g)) != LR_OK) return st;
    if (s->pol_beam && g->npol != 4)
        return fail(LR_E_ARG, "a polarised beam needs npol = 4 (XX, XY, YX, YY)");
    G.n_kind = n_kind_of(s->pol_beam);
    G.h = half_widths(s->n_w, s->h_min, s->h_max);
    G.hmax = *std::max_element(G.h.begin(), G.h.end());
    int32_t smax = 2 * G.hmax + 1;
    G.M = s->screen_m ? s->screen_m : 2 * smax;
    if (G.M <= smax) return fail(LR_E_ARG, "screen_m must exceed the largest support");
    if ((int64_t)G.M > 4096) return fail(LR_E_RANGE, "screen size M must be <= 4096");
    if ((int64_t)s->oversample * G.M > (1 << 20)) return fail(LR_E_RANGE, "O*M too large");
    int64_t no = s->oversample + 1;
    int np = s->n_fg * s->n_w;
    G.plane_off.resize(np);
    int64_t acc = 0;
    for (int f = 0; f < s->n_fg; ++f)
        for (int k = 0; k < s->n_w; ++k) {
            G.plane_off[f * s->n_w + k] = acc;
            int64_t S = 2 * G.h[k] + 1;
            acc += no * no * S * S;
        }
    G.n_elems = acc;
    size_t eb = elem_bytes_of(s->storage);
    G.off_h = 0;
    G.off_po = al256(sizeof(int32_t) * s->n_w);
    G.off_exp = G.off_po + al256(sizeof(int64_t) * np);
    G.off_scale = G.off_exp + al256(sizeof(int32_t) * np * G.n_kind);
    G.off_table = G.off_scale + al256(sizeof(float) * np * G.n_kind);
    // zeroed padding after the table: the paired degridder's loads of a
    // footprint row's last tap may read one element past the table
    G.total = G.off_table + (size_t)G.n_elems * G.n_kind * eb + kTablePad;
    return LR_OK;
}

CFView view_of(const lr_cf *cf) {
    CFView v;
    v.table = cf->d_table;
    v.plane_off = cf->d_plane_off;
    v.scale = cf->d_scale;
    v.h = cf->d_h;
    v.O = cf->spec.oversample;
    v.n_w = cf->spec.n_w;
    v.n_fg = cf->spec.n_fg;
    v.storage = cf->spec.storage;
    // the PS taper alone (and the w = 0 plane) transforms to a real, even
    // kernel: its imaginary parts are rounding noise
    const uint32_t t = cf->spec.terms;
    v.real = !(t & LR_TERM_A) && (!(t & LR_TERM_W) || cf->spec.n_w == 1) ? 1 : 0;
    v.h0 = cf->h[0];
    v.off0 = cf->plane_off[0];
    return v;
}

// The view of one Mueller kind: its table and its planes' scales.
CFView view_kind(const lr_cf *cf, int32_t kind) {
    CFView v = view_of(cf);
    v.table = (const char *)cf->d_table + (size_t)kind * cf->kind_elems * cf->elem_bytes;
    v.scale = cf->d_scale + (size_t)kind * cf->spec.n_fg * cf->spec.n_w;
    return v;
}

lr_cf *make_handle(const lr_cf_spec *s, const lr_grid_spec *g, const Geometry &G, void *buf) {
    lr_cf *cf = new (std::nothrow) lr_cf;
    if (!cf) return nullptr;
    cf->spec = *s;
    cf->fg_hz.assign(s->fg_hz, s->fg_hz + s->n_fg);
    cf->spec.fg_hz = cf->fg_hz.data();
    cf->grid = *g;
    cf->M = G.M;
    cf->h = G.h;
    cf->plane_off = G.plane_off;
    cf->n_kind = G.n_kind;
    cf->kind_elems = G.n_elems;
    cf->n_elems = G.n_elems * G.n_kind;
    kind_map(s->pol_beam, g->npol, cf->kind_of);
    cf->elem_bytes = elem_bytes_of(s->storage);
    cf->header_bytes = G.off_table;
    cf->total_bytes = G.total;
    cf->blob = (char *)buf;
    cf->d_h = (int32_t *)(cf->blob + G.off_h);
    cf->d_plane_off = (int64_t *)(cf->blob + G.off_po);
    cf->d_exp = (int32_t *)(cf->blob + G.off_exp);
    cf->d_scale = (float *)(cf->blob + G.off_scale);
    cf->d_table = cf->blob + G.off_table;
    return cf;
}

// ---- visibility descriptors ----------------------------------------------------
lr_status check_vis(const lr_cf *cf, const lr_vis *v, bool need_vis, bool need_weight) {
    if (!cf) return fail(LR_E_ARG, "cf handle is NULL");
    if (!v) return fail(LR_E_ARG, "vis descriptor is NULL");
    if (v->nrow < 0) return fail(LR_E_ARG, "nrow must be >= 0");
    if (v->nchan < 1) return fail(LR_E_ARG, "nchan must be >= 1");
    if (v->npol != cf->grid.npol) return fail(LR_E_ARG, "vis npol %d != grid npol %d", v->npol, cf->grid.npol);
    if ((int64_t)v->nrow * v->nchan >= (1ll << 30))
        return fail(LR_E_RANGE, "nrow * nchan must be < 2^30 per call (stream larger data in chunks)");
    if (v->nrow > 0 && !v->uvw) return fail(LR_E_ARG, "uvw is NULL");
    if (!v->freq_hz || !v->chan_plane) return fail(LR_E_ARG, "freq_hz and chan_plane are required");
    for (int c = 0; c < v->nchan; ++c) {
        if (!(v->freq_hz[c] > 0.0) || !std::isfinite(v->freq_hz[c]))
            return fail(LR_E_ARG, "freq_hz[%d] must be positive", c);
        if (v->chan_plane[c] >= cf->grid.nplane)
            return fail(LR_E_ARG, "chan_plane[%d] = %d >= nplane", c, v->chan_plane[c]);
        int fg = v->chan_fg ? v->chan_fg[c] : 0;
        if (fg < 0 || fg >= cf->spec.n_fg) return fail(LR_E_ARG, "chan_fg[%d] out of range", c);
    }
    if (need_vis && v->nrow > 0 && !v->vis) return fail(LR_E_ARG, "vis is NULL");
    if (((uintptr_t)v->vis | (uintptr_t)v->weight | (uintptr_t)v->uvw) & 15)
        return fail(LR_E_ARG, "uvw, vis and weight must be 16-byte aligned");
    if (need_weight && v->nrow > 0 && !v->weight) return fail(LR_E_ARG, "weight is NULL");
    bool po = v->ant1 || v->ant2 || v->ant_dlm;
    if (po && !(v->ant1 && v->ant2 && v->ant_dlm && v->nant > 0))
        return fail(LR_E_ARG, "pointing phasor needs ant1, ant2, ant_dlm and nant > 0");
    if (po && (int64_t)v->nant * v->nant > (1 << 24)) return fail(LR_E_RANGE, "nant too large");
    return LR_OK;
}

lr_status check_precision(const lr_cf *cf, lr_precision p) {
    if (elem_bytes_of(p) == 0) return fail(LR_E_DTYPE, "unknown precision %d", (int)p);
    if (cf->spec.storage != p)
        return fail(LR_E_DTYPE, "CF storage %d does not match precision %d",
                    (int)cf->spec.storage, (int)p);
    return LR_OK;
}

std::vector<ChanConst> chan_consts(const lr_cf *cf, const lr_vis *v) {
    std::vector<ChanConst> cc(v->nchan);
    const lr_grid_spec &g = cf->grid;
    const lr_cf_spec &s = cf->spec;
    for (int c = 0; c < v->nchan; ++c) {
        double sc = v->freq_hz[c] / kCLight;
        cc[c].kx = ((sc * (double)g.nx) * g.cell_l) * (double)s.oversample;
        cc[c].ky = ((sc * (double)g.ny) * g.cell_m) * (double)s.oversample;
        cc[c].kw = s.n_w > 1 ? sc * ((double)(s.n_w - 1) / s.w_max) : 0.0;
        cc[c].fscale = ((M_PI * s.dish_m) * v->freq_hz[c]) / kCLight;
        cc[c].plane = v->chan_plane[c];
        cc[c].fg = v->chan_fg ? v->chan_fg[c] : 0;
        cc[c].pad0 = cc[c].pad1 = 0;
    }
    return cc;
}

MapGeom map_geom(const lr_cf *cf, int32_t nchan, int psf) {
    MapGeom m;
    const lr_grid_spec &g = cf->grid;
    m.nx = g.nx;
    m.ny = g.ny;
    m.O = cf->spec.oversample;
    m.n_w = cf->spec.n_w;
    m.psf = psf;
    m.npol = g.npol;
    m.nplane = g.nplane;
    m.nchan = nchan;
    m.ox = (double)(g.nx / 2) * (double)m.O + 0.5;
    m.oy = (double)(g.ny / 2) * (double)m.O + 0.5;
    m.limx = (double)g.nx * (double)m.O;
    m.limy = (double)g.ny * (double)m.O;
    m.h = cf->d_h;
    return m;
}

// (tile, group) pairs per gridder workgroup
int32_t chunk_pairs() {
    static int32_t v = [] {
        const char *e = getenv("LR_TILE_CHUNK");
        int x = e ? atoi(e) : 0;
        return x >= 1 && x <= kChunkMax ? x : kChunkMax;
    }();
    return v;
}

int32_t h_max_of(const lr_cf *cf) { return *std::max_element(cf->h.begin(), cf->h.end()); }

KeyLayout key_layout(const lr_cf *cf, const lr_vis *v, bool po, int32_t &merged) {
    KeyLayout k;
    const lr_grid_spec &g = cf->grid;
    k.b_plane = bitwidth(g.nplane - 1);
    k.b_fg = bitwidth(cf->spec.n_fg - 1);
    k.b_k = bitwidth(cf->spec.n_w - 1);
    k.b_conj = cf->spec.n_w > 1 ? 1 : 0;
    k.b_pv = bitwidth(g.ny - 1);
    k.b_pu = bitwidth(g.nx - 1);
    k.b_bl = po ? bitwidth((int64_t)v->nant * v->nant - 1) : 0;
    k.b_ch = po ? bitwidth(v->nchan - 1) : 0;
    k.b_o = bitwidth(cf->spec.oversample - 1);
    int total = k.b_plane + k.b_fg + k.b_k + k.b_conj + k.b_pv + k.b_pu + k.b_bl + k.b_ch + 2 * k.b_o;
    if (total <= 63) {
        k.shift = 0;
        k.end_bit = total + 1;
        merged = 1;
    } else {
        k.shift = total - 63;
        k.end_bit = 64;
        merged = 0;
    }
    return k;
}

size_t plan_total(const lr_cf *cf, const lr_vis *v) {
    return plan_layout((int64_t)v->nrow * v->nchan, v->nchan, h_max_of(cf),
                       tile_count(cf->grid.nx, cf->grid.ny, cf->grid.nplane)).total;
}

lr_status plan_matches(const lr_plan *P, const lr_cf *cf, const lr_vis *v, int psf) {
    if (P->cf != cf) return fail(LR_E_ARG, "plan was built for another CF handle");
    if (P->nrow != v->nrow || P->nchan != v->nchan || P->npol != v->npol)
        return fail(LR_E_ARG, "plan was built for other data dimensions");
    if (P->psf != psf) return fail(LR_E_ARG, "plan footprint rule (psf=%d) does not match the call", P->psf);
    bool po = v->ant1 != nullptr;
    if ((P->po != 0) != po) return fail(LR_E_ARG, "plan pointing-phasor setting does not match the call");
    for (int c = 0; c < v->nchan; ++c) {
        int fg = v->chan_fg ? v->chan_fg[c] : 0;
        if (P->freq[c] != v->freq_hz[c] || P->chan_plane[c] != v->chan_plane[c] ||
            P->chan_fg[c] != fg)
            return fail(LR_E_ARG, "plan was built for other channel settings");
    }
    return LR_OK;
}

// Build a plan into `buf` (caller memory).  Synchronises the stream.
lr_status build_plan(const lr_cf *cf, const lr_vis *v, int psf, void *buf, size_t bytes,
                     hipStream_t s, lr_plan *P) {
    int64_t n_pairs = (int64_t)v->nrow * v->nchan;
    PlanLayout L = plan_layout(n_pairs, v->nchan, h_max_of(cf),
                               tile_count(cf->grid.nx, cf->grid.ny, cf->grid.nplane));
    if (!buf && L.total) return fail(LR_E_ARG, "plan buffer is NULL");
    if (bytes < L.total) return fail(LR_E_WORKSPACE, "plan needs %zu bytes, got %zu", L.total, bytes);
    bool po = v->ant1 != nullptr;
    P->cf = cf;
    P->nrow = v->nrow;
    P->nchan = v->nchan;
    P->npol = v->npol;
    P->psf = psf;
    P->po = po ? 1 : 0;
    P->freq.assign(v->freq_hz, v->freq_hz + v->nchan);
    P->chan_plane.assign(v->chan_plane, v->chan_plane + v->nchan);
    P->chan_fg.resize(v->nchan);
    for (int c = 0; c < v->nchan; ++c) P->chan_fg[c] = v->chan_fg ? v->chan_fg[c] : 0;
    P->n_pairs = n_pairs;
    P->bytes_used = L.total;
    KeyLayout kl = key_layout(cf, v, po, P->merged);
    char *b = (char *)buf;
    std::vector<ChanConst> cc = chan_consts(cf, v);
    ChanConst *d_cc = (ChanConst *)(b + L.chan);
    hipError_t e = upload_chan(cc, d_cc, s);
    if (e != hipSuccess) return dev_fail(e, "channel upload");
    MapGeom g = map_geom(cf, v->nchan, psf);
    double du_dl = 1.0 / ((double)cf->grid.nx * cf->grid.cell_l);
    double dv_dm = 1.0 / ((double)cf->grid.ny * cf->grid.cell_m);
    // largest-first chunk order for kernel tables up to the size of the
    // last-level cache (256 MB)
    // one kind's table is read per gridder pass
    const bool lpt = (size_t)cf->kind_elems * cf->elem_bytes <= ((size_t)256 << 20);
    e = build_plan_device(P, b, L, v->uvw, d_cc, g, kl, view_of(cf), v->ant1, v->ant2,
                          v->nant, v->ant_dlm, du_dl, dv_dm, chunk_pairs(), kChunkCells, lpt, s);
    if (e == hipErrorInvalidValue)
        return fail(LR_E_RANGE, "plan tile table overflow");
    if (e != hipSuccess) return dev_fail(e, "plan build");
    return LR_OK;
}

// Workspace of the deterministic sums of weights.
static size_t det_bytes(int32_t nchan, int32_t npol) {
    return al256((size_t)std::max(nchan, 1) * kDetRowBlocks * npol * sizeof(double));
}

// Workspace of the deterministic group sums: one flag per group and the
// pieces of groups that cross segment edges.
static size_t det_group_bytes(int64_t n_groups, int64_t n_kept, int32_t npol, lr_precision precision) {
    const int64_t n_seg = (std::max<int64_t>(n_kept, 1) + kDetSeg - 1) / kDetSeg;
    return al256((size_t)std::max<int64_t>(n_groups, 1)) +
           al256((size_t)n_seg * 2 * npol * (precision == LR_F64 ? 16 : 8));
}

// Resolve the plan of a call: the caller's, or a transient one at the start
// of the workspace.  Returns the workspace bytes it used.
lr_status resolve_plan(const lr_cf *cf, const lr_vis *v, int psf, void *work,
                       size_t work_bytes, hipStream_t s, lr_plan &tmp, const lr_plan *&P,
                       size_t &used) {
    if (v->plan) {
        lr_status st = plan_matches(v->plan, cf, v, psf);
        if (st != LR_OK) return st;
        P = v->plan;
        used = 0;
        return LR_OK;
    }
    size_t need = plan_total(cf, v);
    if (work_bytes < need) return fail(LR_E_WORKSPACE, "workspace needs %zu bytes for a transient plan, got %zu", need, work_bytes);
    lr_status st = build_plan(cf, v, psf, work, work_bytes, s, &tmp);
    if (st != LR_OK) return st;
    P = &tmp;
    used = al256(need);
    return LR_OK;
}

size_t cplx_bytes(lr_precision p) { return p == LR_F64 ? 16 : 8; }

}  // namespace

// =============================================================================
extern "C" {

const char *lr_status_str(lr_status s) {
    switch (s) {
        case LR_OK: return "LR_OK";
        case LR_E_ARG: return "LR_E_ARG";
        case LR_E_DTYPE: return "LR_E_DTYPE";
        case LR_E_WORKSPACE: return "LR_E_WORKSPACE";
        case LR_E_CF: return "LR_E_CF";
        case LR_E_DEVICE: return "LR_E_DEVICE";
        case LR_E_RANGE: return "LR_E_RANGE";
    }
    return "LR_E_UNKNOWN";
}

const char *lr_last_error(void) { return g_err.c_str(); }

size_t lr_cf_bytes(const lr_cf_spec *spec, const lr_grid_spec *grid) {
    Geometry G;
    if (geometry(spec, grid, G) != LR_OK) return 0;
    return G.total;
}

size_t lr_workspace_bytes(int op, const lr_cf_spec *spec, const lr_grid_spec *grid,
                          const lr_vis *vis, lr_precision precision) {
    Geometry G;
    if (geometry(spec, grid, G) != LR_OK) return 0;
    if (op == LR_OP_CF_BUILD) return cf_work_bytes(G.M, spec->oversample, G.hmax);
    if (!vis) { fail(LR_E_ARG, "vis descriptor is NULL"); return 0; }
    int64_t n_pairs = (int64_t)vis->nrow * vis->nchan;
    size_t plan = vis->plan ? 0 : al256(plan_layout(n_pairs, vis->nchan, G.hmax,
                                                    tile_count(grid->nx, grid->ny,
                                                               grid->nplane)).total);
    int64_t n_groups = vis->plan ? vis->plan->n_groups : n_pairs;
    size_t per = 0;
    if (op == LR_OP_GRID || op == LR_OP_PSF || op == LR_OP_DEGRID)
        per = al256((size_t)std::max<int64_t>(n_groups, 1) * grid->npol * cplx_bytes(precision));
    // partial sums of weights and group flags of the deterministic mode
    if (op == LR_OP_GRID || op == LR_OP_SUMWT) per += det_bytes(vis->nchan, grid->npol);
    if (op == LR_OP_GRID)
        per += det_group_bytes(n_groups, vis->plan ? vis->plan->n_kept : n_pairs, grid->npol,
                               precision);
    return plan + per + 256;
}

lr_status lr_cf_build(const lr_cf_spec *spec, const lr_grid_spec *grid, void *cf_buf,
                      size_t cf_bytes, void *work, size_t work_bytes, lr_stream stream,
                      lr_cf **out) {
    if (!out) return fail(LR_E_ARG, "out is NULL");
    *out = nullptr;
    Geometry G;
    lr_status st = geometry(spec, grid, G);
    if (st != LR_OK) return st;
    if (!cf_buf) return fail(LR_E_ARG, "cf_buf is NULL");
    if (cf_bytes < G.total) return fail(LR_E_WORKSPACE, "CF blob needs %zu bytes, got %zu", G.total, cf_bytes);
    size_t wneed = cf_work_bytes(G.M, spec->oversample, G.hmax);
    if (!work || work_bytes < wneed)
        return fail(LR_E_WORKSPACE, "CF build needs %zu bytes of workspace, got %zu", wneed, work_bytes);
    lr_cf *cf = make_handle(spec, grid, G, cf_buf);
    if (!cf) return fail(LR_E_ARG, "out of host memory");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = upload_words(G.h.data(), sizeof(int32_t) * G.h.size(), cf->d_h, s);
    if (e == hipSuccess)
        e = upload_words(G.plane_off.data(), sizeof(int64_t) * G.plane_off.size(),
                         cf->d_plane_off, s);
    if (e != hipSuccess) { delete cf; return dev_fail(e, "CF header upload"); }
    CFBuildArgs a;
    a.M = G.M;
    a.O = spec->oversample;
    a.nx = grid->nx;
    a.ny = grid->ny;
    a.terms = (int32_t)spec->terms;
    a.cell_l = grid->cell_l;
    a.cell_m = grid->cell_m;
    a.c_ps = M_PI * spec->ps_support / 2.0;
    a.dish_m = spec->dish_m;
    a.pol_beam = spec->pol_beam;
    a.kind = 0;
    a.eta = spec->beam_ellipticity;
    a.kappa = spec->beam_leakage;
    e = launch_cf_build(cf, a, work, s);
    if (e == hipSuccess)
        e = launch_zero((char *)cf->d_table + (size_t)cf->n_elems * cf->elem_bytes, kTablePad, s);
    if (e != hipSuccess) { delete cf; return dev_fail(e, "CF build"); }
    *out = cf;
    return LR_OK;
}

lr_status lr_cf_attach(const lr_cf_spec *spec, const lr_grid_spec *grid, void *cf_buf,
                       size_t cf_bytes, lr_cf **out) {
    if (!out) return fail(LR_E_ARG, "out is NULL");
    *out = nullptr;
    Geometry G;
    lr_status st = geometry(spec, grid, G);
    if (st != LR_OK) return st;
    if (!cf_buf) return fail(LR_E_ARG, "cf_buf is NULL");
    if (cf_bytes < G.total) return fail(LR_E_CF, "CF blob has %zu bytes, the spec needs %zu", cf_bytes, G.total);
    lr_cf *cf = make_handle(spec, grid, G, cf_buf);
    if (!cf) return fail(LR_E_ARG, "out of host memory");
    *out = cf;
    return LR_OK;
}

void lr_cf_free(lr_cf *cf) { delete cf; }

lr_status lr_cf_scale_exponents(const lr_cf *cf, int32_t *exps, lr_stream stream) {
    if (!cf || !exps) return fail(LR_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    size_t n = (size_t)cf->spec.n_fg * cf->spec.n_w * cf->n_kind;
    hipError_t e = hipMemcpyAsync(exps, cf->d_exp, n * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return dev_fail(e, "read scale exponents");
    return LR_OK;
}

lr_status lr_cf_kinds(const lr_cf *cf, int32_t *n_kind, int32_t *kind_of) {
    if (!cf) return fail(LR_E_ARG, "cf handle is NULL");
    if (n_kind) *n_kind = cf->n_kind;
    if (kind_of) std::copy(cf->kind_of, cf->kind_of + 16, kind_of);
    return LR_OK;
}

lr_status lr_cf_layout(const lr_cf *cf, size_t *table_offset, size_t *elem_bytes,
                       int64_t *n_elems, int64_t *plane_off) {
    if (!cf) return fail(LR_E_ARG, "cf handle is NULL");
    if (table_offset) *table_offset = cf->header_bytes;
    if (elem_bytes) *elem_bytes = cf->elem_bytes;
    if (n_elems) *n_elems = cf->n_elems;
    if (plane_off) std::copy(cf->plane_off.begin(), cf->plane_off.end(), plane_off);
    return LR_OK;
}

size_t lr_plan_bytes(const lr_cf *cf, const lr_vis *vis, int psf) {
    (void)psf;
    if (check_vis(cf, vis, false, false) != LR_OK) return 0;
    return plan_total(cf, vis);
}

lr_status lr_plan_build(const lr_cf *cf, const lr_vis *vis, int psf, void *buf, size_t bytes,
                        lr_stream stream, lr_plan **out) {
    if (!out) return fail(LR_E_ARG, "out is NULL");
    *out = nullptr;
    lr_status st = check_vis(cf, vis, false, false);
    if (st != LR_OK) return st;
    lr_plan *P = new (std::nothrow) lr_plan;
    if (!P) return fail(LR_E_ARG, "out of host memory");
    st = build_plan(cf, vis, psf ? 1 : 0, buf, bytes, (hipStream_t)stream, P);
    if (st != LR_OK) { delete P; return st; }
    *out = P;
    return LR_OK;
}

void lr_plan_free(lr_plan *plan) { delete plan; }

namespace {
// The arrays a built plan keeps, at their actual sizes (the build buffer is
// sized for the worst case and also holds the build's transient arrays).
struct PackedLayout {
    size_t chan, order, gidx, pair_group, group_start, groups, tp_group, chunk_start,
        chunk_tile, chunk_excl, chunk_order, tile_state, shared_tiles, geo, tile_tp, multi,
        sep_part, sep_shared, total;
};

PackedLayout packed_layout(const lr_plan *P) {
    PackedLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += al256(bytes); return o; };
    L.chan = take(sizeof(ChanConst) * std::max<int32_t>(P->nchan, 1));
    L.order = take(sizeof(int32_t) * P->n_pairs);
    L.gidx = take(sizeof(int32_t) * P->n_kept);
    L.pair_group = take(sizeof(int32_t) * P->n_pairs);
    L.group_start = take(sizeof(int32_t) * (P->n_groups + 1));
    L.groups = take(sizeof(GroupMeta) * P->n_groups);
    L.tp_group = take(sizeof(int32_t) * P->n_tile_pairs);
    L.chunk_start = take(sizeof(int32_t) * (P->n_chunks + 1));
    L.chunk_tile = take(sizeof(int32_t) * P->n_chunks);
    L.chunk_excl = take(sizeof(int32_t) * P->n_chunks);
    L.chunk_order = take(P->chunk_order ? sizeof(int32_t) * P->n_chunks : 0);
    L.tile_state = take(sizeof(int32_t) * P->n_tiles);
    L.shared_tiles = take(sizeof(int32_t) * P->n_shared);
    L.geo = take(sizeof(int64_t) * P->n_groups);
    L.tile_tp = take(sizeof(int32_t) * (P->n_tiles + 1));
    L.multi = take(sizeof(int32_t) * P->n_multi);
    L.sep_part = take(sizeof(int4) * P->n_sep_parts);
    L.sep_shared = take(sizeof(int32_t) * P->n_sep_shared);
    L.total = off;
    return L;
}
}  // namespace

size_t lr_plan_packed_bytes(const lr_plan *plan) {
    if (!plan) { fail(LR_E_ARG, "plan is NULL"); return 0; }
    return packed_layout(plan).total;
}

lr_status lr_plan_pack(const lr_plan *plan, void *buf, size_t bytes, lr_stream stream,
                       lr_plan **out) {
    if (!out) return fail(LR_E_ARG, "out is NULL");
    *out = nullptr;
    if (!plan) return fail(LR_E_ARG, "plan is NULL");
    const PackedLayout L = packed_layout(plan);
    if (!buf) return fail(LR_E_ARG, "buf is NULL");
    if (bytes < L.total) return fail(LR_E_WORKSPACE, "packed plan needs %zu bytes, got %zu", L.total, bytes);
    lr_plan *Q = new (std::nothrow) lr_plan(*plan);
    if (!Q) return fail(LR_E_ARG, "out of host memory");
    hipStream_t s = (hipStream_t)stream;
    char *b = (char *)buf;
    hipError_t e = hipSuccess;
    auto move = [&](auto *&dst, const void *src, size_t off, size_t n_bytes) {
        using Ptr = typename std::remove_reference<decltype(dst)>::type;
        dst = (Ptr)(b + off);
        if (e == hipSuccess && n_bytes)
            e = hipMemcpyAsync(b + off, src, n_bytes, hipMemcpyDeviceToDevice, s);
    };
    const lr_plan *P = plan;
    move(Q->cc, P->cc, L.chan, sizeof(ChanConst) * P->nchan);
    move(Q->order, P->order, L.order, sizeof(int32_t) * P->n_pairs);
    move(Q->gidx, P->gidx, L.gidx, sizeof(int32_t) * P->n_kept);
    move(Q->pair_group, P->pair_group, L.pair_group, sizeof(int32_t) * P->n_pairs);
    move(Q->group_start, P->group_start, L.group_start, sizeof(int32_t) * (P->n_groups + 1));
    move(Q->groups, P->groups, L.groups, sizeof(GroupMeta) * P->n_groups);
    move(Q->tp_group, P->tp_group, L.tp_group, sizeof(int32_t) * P->n_tile_pairs);
    move(Q->chunk_start, P->chunk_start, L.chunk_start, sizeof(int32_t) * (P->n_chunks + 1));
    move(Q->chunk_tile, P->chunk_tile, L.chunk_tile, sizeof(int32_t) * P->n_chunks);
    move(Q->chunk_excl, P->chunk_excl, L.chunk_excl, sizeof(int32_t) * P->n_chunks);
    if (P->chunk_order)
        move(Q->chunk_order, P->chunk_order, L.chunk_order, sizeof(int32_t) * P->n_chunks);
    move(Q->tile_state, P->tile_state, L.tile_state, sizeof(int32_t) * P->n_tiles);
    move(Q->shared_tiles, P->shared_tiles, L.shared_tiles, sizeof(int32_t) * P->n_shared);
    move(Q->geo, P->geo, L.geo, sizeof(int64_t) * P->n_groups);
    move(Q->tile_tp, P->tile_tp, L.tile_tp, sizeof(int32_t) * (P->n_tiles + 1));
    move(Q->multi, P->multi, L.multi, sizeof(int32_t) * P->n_multi);
    move(Q->sep_part, P->sep_part, L.sep_part, sizeof(int4) * P->n_sep_parts);
    move(Q->sep_shared, P->sep_shared, L.sep_shared, sizeof(int32_t) * P->n_sep_shared);
    Q->bytes_used = L.total;
    if (e != hipSuccess) { delete Q; return dev_fail(e, "plan pack"); }
    *out = Q;
    return LR_OK;
}

lr_status lr_gcf(const lr_cf *cf, int32_t fg, int32_t k, int32_t n, void *out,
                 lr_stream stream) {
    if (!cf || !out) return fail(LR_E_ARG, "NULL argument");
    if (n <= 0) return fail(LR_E_ARG, "n must be positive");
    if (fg < 0 || fg >= cf->spec.n_fg || k < 0 || k >= cf->spec.n_w)
        return fail(LR_E_RANGE, "plane (%d, %d) out of range", fg, k);
    if (cf->spec.terms & LR_TERM_A)
        return fail(LR_E_ARG, "grid correction needs a separable plane (no A term)");
    if ((cf->spec.terms & LR_TERM_W) && k != 0 && cf->spec.n_w > 1)
        return fail(LR_E_ARG, "grid correction needs a separable plane (w-plane 0)");
    hipStream_t s = (hipStream_t)stream;
    const size_t i = (size_t)fg * cf->spec.n_w + k;
    float sc = 1.0f;
    if (cf->elem_bytes == 4) {
        int32_t e = 0;
        hipError_t he = hipMemcpyAsync(&e, cf->d_exp + i, sizeof e, hipMemcpyDeviceToHost, s);
        if (he == hipSuccess) he = hipStreamSynchronize(s);
        if (he != hipSuccess) return dev_fail(he, "read plane exponent");
        sc = std::ldexp(1.0f, -e);
    }
    hipError_t e = launch_gcf(view_of(cf), cf->plane_off[i], cf->h[k], sc, n, (double2 *)out, s);
    if (e != hipSuccess) return dev_fail(e, "gcf");
    return LR_OK;
}

lr_status lr_image_normalize(const lr_cf *cf, lr_precision precision, const void *img,
                             const double *gcf_x, const double *gcf_y, const double *sumwt,
                             void *out, lr_stream stream) {
    if (!cf || !img || !gcf_x || !gcf_y || !sumwt || !out) return fail(LR_E_ARG, "NULL argument");
    if (precision < LR_F64 || precision > LR_F32_CFBF16) return fail(LR_E_DTYPE, "bad precision");
    const lr_grid_spec &g = cf->grid;
    hipError_t e = launch_normalize(img, gcf_x, gcf_y, sumwt, g.nx, g.ny,
                                    (int64_t)g.nplane * g.npol, precision, out,
                                    (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "image normalisation");
    return LR_OK;
}

lr_status lr_ps_taper(const lr_cf *cf, int32_t n, void *out, lr_stream stream) {
    if (!cf || !out) return fail(LR_E_ARG, "NULL argument");
    if (n <= 0) return fail(LR_E_ARG, "n must be positive");
    const int use_ps = (cf->spec.terms & LR_TERM_PS) ? 1 : 0;
    hipError_t e = launch_ps_taper(M_PI * cf->spec.ps_support / 2.0, use_ps, n, (double *)out,
                                   (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "PS taper");
    return LR_OK;
}

lr_status lr_pb_image(const lr_cf *cf, const double *fg_weight, void *out, lr_stream stream) {
    if (!cf || !fg_weight || !out) return fail(LR_E_ARG, "NULL argument");
    if (cf->n_kind > 1)
        return fail(LR_E_CF, "the weight image is defined for a scalar beam (pol_beam = 0)");
    hipError_t e = launch_pb_image(cf, fg_weight, (double *)out, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "weight image");
    return LR_OK;
}

lr_status lr_image_normalize_pb(const lr_cf *cf, lr_precision precision, const void *img,
                                const double *gcf_x, const double *gcf_y, const double *sumwt,
                                const double *pb, double pb_min, void *out, lr_stream stream) {
    if (!cf || !img || !gcf_x || !gcf_y || !sumwt || !pb || !out)
        return fail(LR_E_ARG, "NULL argument");
    if (precision < LR_F64 || precision > LR_F32_CFBF16) return fail(LR_E_DTYPE, "bad precision");
    if (!(pb_min > 0.0)) return fail(LR_E_ARG, "pb_min must be positive");
    const lr_grid_spec &g = cf->grid;
    hipError_t e = launch_normalize_pb(img, gcf_x, gcf_y, sumwt, pb, pb_min, g.nx, g.ny,
                                       (int64_t)g.nplane * g.npol, precision, out,
                                       (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "image normalisation");
    return LR_OK;
}

size_t lr_hogbom_work_bytes(int32_t nx, int32_t ny) {
    if (nx <= 0 || ny <= 0) { fail(LR_E_ARG, "image size must be positive"); return 0; }
    return hogbom_work_bytes(nx, ny);
}

lr_status lr_hogbom(const void *psf, void *residual, void *model, int32_t nx, int32_t ny,
                    lr_precision precision, double gain, double threshold, int32_t niter,
                    int32_t *iterations, void *work, size_t work_bytes, lr_stream stream) {
    if (!psf || !residual || !model || !iterations || !work)
        return fail(LR_E_ARG, "NULL argument");
    if (nx <= 0 || ny <= 0) return fail(LR_E_ARG, "image size must be positive");
    if (precision != LR_F64 && precision != LR_F32)
        return fail(LR_E_DTYPE, "images are float64 (LR_F64) or float32 (LR_F32)");
    if (!(gain > 0.0 && gain <= 1.0)) return fail(LR_E_ARG, "gain must be in (0, 1]");
    if (niter < 0) return fail(LR_E_ARG, "niter must be >= 0");
    if (work_bytes < hogbom_work_bytes(nx, ny))
        return fail(LR_E_WORKSPACE, "workspace needs %zu bytes, got %zu",
                    hogbom_work_bytes(nx, ny), work_bytes);
    hipError_t e = launch_hogbom(residual, psf, model, nx, ny, precision, gain, threshold,
                                 niter, work, iterations, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "hogbom");
    return LR_OK;
}

lr_status lr_rephase(int64_t nrow, int32_t nchan, int32_t npol, lr_precision precision,
                     void *vis, const double *uvw, const double *freq_hz, const int32_t *field,
                     const double *field_dlm, int32_t nfield, int32_t direction,
                     lr_stream stream) {
    if (precision != LR_F64 && precision != LR_F32)
        return fail(LR_E_DTYPE, "visibilities are complex128 (LR_F64) or complex64 (LR_F32)");
    if (nrow < 0 || nchan < 0 || npol < 1 || nfield < 0)
        return fail(LR_E_ARG, "negative size");
    if (nrow == 0 || nchan == 0 || nfield == 0) return LR_OK;
    if (!vis || !uvw || !freq_hz || !field || !field_dlm) return fail(LR_E_ARG, "NULL argument");
    hipError_t e = launch_rephase(vis, uvw, freq_hz, field, field_dlm, nrow, nchan, npol, nfield,
                                  (int)precision, direction, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "rephase");
    return LR_OK;
}

lr_status lr_cal_vavg(int64_t nrow, int32_t nchan, int32_t npol, lr_precision precision,
                      const void *vis_obs, const void *vis_model, const void *weight,
                      const int32_t *ant1, const int32_t *ant2, int32_t nant,
                      const int32_t *row_sol, int32_t n_tsol, const int32_t *chan_sol,
                      int32_t n_fsol, int32_t rows_per_step, double *X, double *w,
                      lr_stream stream) {
    if (precision != LR_F64 && precision != LR_F32)
        return fail(LR_E_DTYPE, "visibilities are complex128 (LR_F64) or complex64 (LR_F32)");
    if (!X || !w || !chan_sol) return fail(LR_E_ARG, "NULL argument");
    if (nrow > 0 && (!vis_obs || !vis_model || !ant1 || !ant2 || !row_sol))
        return fail(LR_E_ARG, "NULL argument");
    if (nrow < 0 || nchan < 1 || (npol != 1 && npol != 2 && npol != 4))
        return fail(LR_E_ARG, "bad shape nrow %lld nchan %d npol %d", (long long)nrow, nchan, npol);
    if (nant < 1 || nant > 65535 || n_tsol < 1 || n_fsol < 1 || rows_per_step < 1)
        return fail(LR_E_ARG, "nant, interval counts and rows_per_step must be positive");
    const int64_t npar = npol == 1 ? 1 : 2;
    const double cells = (double)n_tsol * n_fsol * npar * nant * nant;
    if (cells > 4.0e9) return fail(LR_E_ARG, "output of %.3g matrix cells is too large", cells);
    CalVavg c{vis_obs, vis_model, weight, ant1, ant2, row_sol, chan_sol, nrow, nchan, npol,
              nant, n_tsol, n_fsol, rows_per_step, (int32_t)precision, X, w};
    hipError_t e = launch_cal_vavg(c, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "cal_vavg");
    return LR_OK;
}

lr_status lr_cal_solve(const double *X, const double *w, int32_t nant, int64_t n_problems,
                       double alpha, double delta, int32_t max_iter, double *g,
                       int32_t *iterations, double *change, lr_stream stream) {
    if (!X || !w || !g || !iterations || !change) return fail(LR_E_ARG, "NULL argument");
    if (nant < 1 || nant > 2048) return fail(LR_E_ARG, "nant must be in [1, 2048]");
    if (n_problems < 0 || n_problems > 0x7fffffff) return fail(LR_E_ARG, "bad n_problems");
    if (!(alpha > 0.0 && alpha <= 1.0)) return fail(LR_E_ARG, "alpha must be in (0, 1]");
    if (!(delta >= 0.0) || max_iter < 0) return fail(LR_E_ARG, "delta < 0 or max_iter < 0");
    hipError_t e = launch_cal_solve(X, w, nant, n_problems, alpha, delta, max_iter, g,
                                    iterations, change, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "cal_solve");
    return LR_OK;
}

lr_status lr_plan_info(const lr_plan *plan, int64_t *n_groups, int64_t *n_kept,
                       int64_t *n_pairs, int64_t *taps) {
    if (!plan) return fail(LR_E_ARG, "plan is NULL");
    if (n_groups) *n_groups = plan->n_groups;
    if (n_kept) *n_kept = plan->n_kept;
    if (n_pairs) *n_pairs = plan->n_pairs;
    if (taps) *taps = plan->taps;
    return LR_OK;
}

lr_status lr_set_deterministic(int32_t on) {
    g_det.store(on ? 1 : 0);
    return LR_OK;
}

int32_t lr_deterministic(void) { return g_det.load(); }

lr_status lr_set_profile_events(void *start, void *stop) {
    if ((start == nullptr) != (stop == nullptr))
        return fail(LR_E_ARG, "give both events or neither");
    g_prof_start = (hipEvent_t)start;
    g_prof_stop = (hipEvent_t)stop;
    return LR_OK;
}

// Scratch of a gridding call beyond a transient plan: the group sums and,
// in the deterministic order, its partial sums.  a_bytes receives the
// group-sum part.
static size_t grid_scratch_bytes(const lr_vis *vis, lr_precision precision, bool det,
                                 size_t &a_bytes) {
    int64_t ng_bound = vis->plan ? vis->plan->n_groups : (int64_t)vis->nrow * vis->nchan;
    a_bytes = al256((size_t)std::max<int64_t>(ng_bound, 1) * vis->npol * cplx_bytes(precision));
    const size_t d_bytes =
        det ? det_bytes(vis->nchan, vis->npol) +
                  det_group_bytes(ng_bound,
                                  vis->plan ? vis->plan->n_kept : (int64_t)vis->nrow * vis->nchan,
                                  vis->npol, precision)
            : 0;
    return a_bytes + d_bytes;
}

// Fixed device scratch of lr_grid_static, one copy per GPU the library runs
// on, held until the process ends.  Host code never passes `scratch` itself
// (on the host it is only a stand-in for the symbol): the device address of
// each GPU's copy comes from hipGetSymbolAddress with that GPU current, once
// per device, and only that address reaches kernels.
static constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices];
}  // namespace

// Device address of the current GPU's copy of `scratch`.
static lr_status static_scratch(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return dev_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(LR_E_DEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return dev_fail(e, "scratch symbol address");
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return LR_OK;
}

// The gridder launches of one call: one for a scalar beam; one per Mueller
// kind otherwise, each with its table and the mask that sums the
// correlations of its elements into their grid pols (the first pass may
// write a fresh grid, the later ones add).
static hipError_t grid_passes(const lr_cf *cf, const lr_plan *P, const void *A, void *grid,
                              lr_precision precision, int32_t npol, int mode, bool det,
                              hipStream_t s) {
    if (cf->n_kind == 1)
        return launch_grid(P, view_of(cf), A, grid, precision, npol, cf->grid.nx, cf->grid.ny,
                           mode, det, 0u, s);
    hipError_t e = hipSuccess;
    for (int32_t kind = 0; kind < cf->n_kind && e == hipSuccess; ++kind) {
        const int m = (kind > 0 && mode == GRID_SET) ? GRID_ADD : mode;
        e = launch_grid(P, view_kind(cf, kind), A, grid, precision, npol, cf->grid.nx,
                        cf->grid.ny, m, det, kind_mask(cf, kind, npol), s);
    }
    return e;
}

static lr_status grid_common(const lr_cf *cf, const lr_vis *vis, lr_precision precision,
                             void *grid, double *sumwt, int64_t *counters, void *work,
                             size_t work_bytes, lr_stream stream, int mode) {
    const int psf = mode == GRID_PSF ? 1 : 0;
    lr_status st = check_vis(cf, vis, !psf, true);
    if (st != LR_OK) return st;
    if (psf && cf->n_kind > 1)
        return fail(LR_E_CF, "the PSF takes a table of one scalar beam (pol_beam = 0)");
    if ((st = check_precision(cf, precision)) != LR_OK) return st;
    if (!grid) return fail(LR_E_ARG, "grid is NULL");
    if (!work && work_bytes) return fail(LR_E_ARG, "work is NULL");
    hipStream_t s = (hipStream_t)stream;
    // size check of the per-call scratch before anything is enqueued
    int64_t ng_bound = vis->plan ? vis->plan->n_groups : (int64_t)vis->nrow * vis->nchan;
    size_t plan_need = vis->plan ? 0 : al256(plan_total(cf, vis));
    // deterministic order (lr_set_deterministic): not for the PSF
    const bool det = g_det.load() != 0 && !psf;
    size_t a_bytes = 0;
    const size_t scratch_need = grid_scratch_bytes(vis, precision, det, a_bytes);
    if (work_bytes < plan_need + scratch_need)
        return fail(LR_E_WORKSPACE, "workspace needs %zu bytes, got %zu",
                    plan_need + scratch_need, work_bytes);
    lr_plan tmp;
    const lr_plan *P = nullptr;
    size_t used = 0;
    if ((st = resolve_plan(cf, vis, psf, work, work_bytes, s, tmp, P, used)) != LR_OK) return st;
    void *A = (char *)work + used;
    VisArgs va{vis->vis, vis->weight, vis->npol, psf ? 1 : 0};
    ProfileScope prof(s);
    // group sums start at zero; GRID_SET replaces the outputs, so it also
    // clears sumwt, the counters and the shared tiles
    const bool set = mode == GRID_SET;
    if (det) {
        // every sum in a fixed order: group sums stored per group, sums of
        // weights from fixed partials, one workgroup per tile
        double *part = (double *)((char *)A + a_bytes);
        uint8_t *done = (uint8_t *)part + det_bytes(vis->nchan, vis->npol);
        void *pieces = done + al256((size_t)std::max<int64_t>(ng_bound, 1));
        hipError_t e = launch_grid_setup(P, nullptr, 0, set ? sumwt : nullptr,
                                         sizeof(double) * cf->grid.nplane * vis->npol,
                                         set ? counters : nullptr, grid, precision, vis->npol,
                                         cf->grid.nx, cf->grid.ny, set, false, s);
        if (e == hipSuccess && sumwt)
            e = launch_sumwt_det(P, vis->weight, precision, vis->npol, cf->grid.nplane, part,
                                 sumwt, s);
        if (e == hipSuccess)
            e = launch_presum_det(P, va, precision, A, done, pieces, counters, s);
        if (e == hipSuccess) {
            prof.begin();
            e = grid_passes(cf, P, A, grid, precision, vis->npol, mode, true, s);
            prof.end();
        }
        if (e != hipSuccess) return dev_fail(e, "grid");
        return LR_OK;
    }
    // the separable small-support gridder writes whole tiles itself; only
    // tiles it splits into several parts are cleared first (GRID_SET)
    const CFView view = view_of(cf);
    const bool sep = sep_gridder(P, view, mode, false);
    hipError_t e = launch_grid_setup(
        P, A, (size_t)P->n_groups * vis->npol * cplx_bytes(precision), set ? sumwt : nullptr,
        sizeof(double) * cf->grid.nplane * vis->npol, set ? counters : nullptr, grid, precision,
        vis->npol, cf->grid.nx, cf->grid.ny, set, sep, s);
    if (e == hipSuccess)
        e = launch_presum(P, va, precision, A, sumwt, counters, cf->grid.nplane, s);
    if (e == hipSuccess) {
        prof.begin();
        e = grid_passes(cf, P, A, grid, precision, vis->npol, mode, false, s);
        prof.end();
    }
    if (e != hipSuccess) return dev_fail(e, psf ? "psf" : "grid");
    return LR_OK;
}

lr_status lr_grid(const lr_cf *cf, const lr_vis *vis, lr_precision precision, void *grid,
                  double *sumwt, int64_t *counters, void *work, size_t work_bytes,
                  lr_stream stream) {
    return grid_common(cf, vis, precision, grid, sumwt, counters, work, work_bytes, stream,
                       GRID_ADD);
}

lr_status lr_grid_overwrite(const lr_cf *cf, const lr_vis *vis, lr_precision precision,
                            void *grid, double *sumwt, int64_t *counters, void *work,
                            size_t work_bytes, lr_stream stream) {
    return grid_common(cf, vis, precision, grid, sumwt, counters, work, work_bytes, stream,
                       GRID_SET);
}

lr_status lr_grid_static(const lr_cf *cf, const lr_vis *vis, lr_precision precision,
                         void *grid, double *sumwt, int64_t *counters, lr_stream stream) {
    if (!vis) return fail(LR_E_ARG, "vis descriptor is NULL");
    if (!vis->plan)
        return fail(LR_E_ARG, "lr_grid_static needs a binning plan (vis->plan): a transient "
                              "plan would need workspace");
    if (vis->npol < 1 || vis->npol > 4) return fail(LR_E_ARG, "npol must be 1, 2 or 4");
    size_t a_bytes = 0;
    const size_t need = grid_scratch_bytes(vis, precision, g_det.load() != 0, a_bytes);
    if (need > kStaticScratchBytes)
        return fail(LR_E_RANGE, "lr_grid_static: this plan needs %zu bytes of scratch, beyond "
                                "the library's fixed %zu (%lld groups x %d pols); use lr_grid",
                    need, kStaticScratchBytes, (long long)vis->plan->n_groups, vis->npol);
    void *work = nullptr;
    lr_status st = static_scratch(&work);
    if (st != LR_OK) return st;
    return grid_common(cf, vis, precision, grid, sumwt, counters, work, kStaticScratchBytes,
                       stream, GRID_ADD);
}

lr_status lr_make_psf(const lr_cf *cf, const lr_vis *vis, lr_precision precision,
                      void *psf_grid, double *sumwt, int64_t *counters, void *work,
                      size_t work_bytes, lr_stream stream) {
    return grid_common(cf, vis, precision, psf_grid, sumwt, counters, work, work_bytes, stream,
                       GRID_PSF);
}

lr_status lr_degrid(const lr_cf *cf, lr_vis *vis, lr_precision precision, const void *grid,
                    int64_t *counters, void *work, size_t work_bytes, lr_stream stream) {
    lr_status st = check_vis(cf, vis, true, false);
    if (st != LR_OK) return st;
    if ((st = check_precision(cf, precision)) != LR_OK) return st;
    if (!grid) return fail(LR_E_ARG, "grid is NULL");
    hipStream_t s = (hipStream_t)stream;
    int64_t ng_bound = vis->plan ? vis->plan->n_groups : (int64_t)vis->nrow * vis->nchan;
    size_t v_bytes = al256((size_t)std::max<int64_t>(ng_bound, 1) * vis->npol * cplx_bytes(precision));
    size_t plan_need = vis->plan ? 0 : al256(plan_total(cf, vis));
    if (work_bytes < plan_need + v_bytes)
        return fail(LR_E_WORKSPACE, "workspace needs %zu bytes, got %zu", plan_need + v_bytes, work_bytes);
    lr_plan tmp;
    const lr_plan *P = nullptr;
    size_t used = 0;
    if ((st = resolve_plan(cf, vis, 0, work, work_bytes, s, tmp, P, used)) != LR_OK) return st;
    void *Vg = (char *)work + used;
    ProfileScope prof(s);
    prof.begin();
    hipError_t e = hipSuccess;
    if (cf->n_kind == 1) {
        e = launch_degrid(P, view_of(cf), grid, Vg, precision, vis->npol, cf->grid.nx,
                          cf->grid.ny, h_max_of(cf), 0u, false, s);
    } else {
        // one pass per Mueller kind, each adding its elements' gathers
        for (int32_t kind = 0; kind < cf->n_kind && e == hipSuccess; ++kind)
            e = launch_degrid(P, view_kind(cf, kind), grid, Vg, precision, vis->npol,
                              cf->grid.nx, cf->grid.ny, h_max_of(cf),
                              kind_mask(cf, kind, vis->npol), kind > 0, s);
    }
    prof.end();
    if (e == hipSuccess) e = launch_expand(P, Vg, vis->vis, vis->weight, precision, vis->npol, s);
    if (e == hipSuccess && counters)
        e = launch_counts(P, vis->weight, precision, vis->npol, nullptr, counters,
                          cf->grid.nplane, s);
    if (e != hipSuccess) return dev_fail(e, "degrid");
    return LR_OK;
}

lr_status lr_sumwt(const lr_cf *cf, const lr_vis *vis, lr_precision precision, double *sumwt,
                   int64_t *counters, void *work, size_t work_bytes, lr_stream stream) {
    lr_status st = check_vis(cf, vis, false, true);
    if (st != LR_OK) return st;
    if ((st = check_precision(cf, precision)) != LR_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    lr_plan tmp;
    const lr_plan *P = nullptr;
    size_t used = 0;
    if ((st = resolve_plan(cf, vis, 0, work, work_bytes, s, tmp, P, used)) != LR_OK) return st;
    const bool det = g_det.load() != 0;
    if (det && work_bytes < used + det_bytes(vis->nchan, vis->npol))
        return fail(LR_E_WORKSPACE, "workspace needs %zu bytes, got %zu",
                    used + det_bytes(vis->nchan, vis->npol), work_bytes);
    hipError_t e = launch_counts(P, vis->weight, precision, vis->npol, det ? nullptr : sumwt,
                                 counters, cf->grid.nplane, s);
    if (e == hipSuccess && det && sumwt)
        e = launch_sumwt_det(P, vis->weight, precision, vis->npol, cf->grid.nplane,
                             (double *)((char *)work + used), sumwt, s);
    if (e != hipSuccess) return dev_fail(e, "sumwt");
    return LR_OK;
}

lr_status lr_debug_map(const lr_cf *cf, const lr_vis *vis, int psf, int32_t *out,
                       lr_stream stream) {
    lr_status st = check_vis(cf, vis, false, false);
    if (st != LR_OK) return st;
    if (!out && vis->nrow > 0) return fail(LR_E_ARG, "out is NULL");
    std::vector<ChanConst> cc = chan_consts(cf, vis);
    MapGeom g = map_geom(cf, vis->nchan, psf ? 1 : 0);
    hipError_t e = launch_debug_map(vis->nrow, vis->nchan, vis->uvw, cc, g, out,
                                    (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "debug map");
    return LR_OK;
}

}  // extern "C"
