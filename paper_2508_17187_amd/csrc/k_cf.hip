// Convolution-function construction on the GPU (the ConvFunc component and
// the CFCache's PreCompute step; Table AWP-CFSETUP for the term products).
//
//   taper   psi_0(c, eta) from the prolate spheroidal differential equation:
//           in the basis of normalised even Legendre polynomials the operator
//           -(d/dx)(1 - x^2)(d/dx) + c^2 x^2 is symmetric tridiagonal; its
//           smallest eigenvalue (bisection on Sturm counts) and eigenvector
//           (shifted inverse iteration) give the Legendre coefficients.
//   screen  a_i a_j T(l_j) T(m_i) [B(rho)] [W_k] on (M+1)^2 points.
//   kernel  only the (O S + 1)^2 uv points the table needs, by a separable
//           partial DFT of length O M with exactly reduced integer phases:
//           pass 1 over l for every needed n_u, pass 2 over m for every
//           needed n_v.  No full O M x O M transform is formed.
//   table   conj K / M^2 at (o_u - O t_u, o_v - O t_v), stored as f64, f32,
//           or fp16 / bf16 scaled by 2^e per plane (round to nearest even).
#include "lr_internal.h"
#include "lr_launch.h"

namespace lr {

constexpr int kLegTerms = 48;

__device__ void pswf_coef(double c, double *coef) {
    double d[kLegTerms], e[kLegTerms], x[kLegTerms], y[kLegTerms], wk[kLegTerms];
    const double c2 = c * c;
    for (int k = 0; k < kLegTerms; ++k) {
        double n = 2.0 * k;
        d[k] = n * (n + 1.0) + c2 * (2.0 * n * n + 2.0 * n - 1.0) / ((2.0 * n - 1.0) * (2.0 * n + 3.0));
        e[k] = c2 * (n + 1.0) * (n + 2.0) / ((2.0 * n + 3.0) * sqrt((2.0 * n + 1.0) * (2.0 * n + 5.0)));
    }
    // Gershgorin interval
    double lo = 1e300, hi = -1e300;
    for (int k = 0; k < kLegTerms; ++k) {
        double r = (k > 0 ? fabs(e[k - 1]) : 0.0) + (k < kLegTerms - 1 ? fabs(e[k]) : 0.0);
        lo = fmin(lo, d[k] - r);
        hi = fmax(hi, d[k] + r);
    }
    // bisection for the smallest eigenvalue: count of eigenvalues below mid
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        int cnt = 0;
        double q = d[0] - mid;
        if (q < 0) ++cnt;
        for (int k = 1; k < kLegTerms; ++k) {
            if (q == 0.0) q = 1e-300;
            q = d[k] - mid - e[k - 1] * e[k - 1] / q;
            if (q < 0) ++cnt;
        }
        if (cnt >= 1) hi = mid; else lo = mid;
    }
    // shifted inverse iteration: T - sigma I is positive definite for sigma
    // below the smallest eigenvalue, so elimination without pivoting is stable
    double sigma = lo - 1e-10 * fmax(1.0, fabs(lo));
    for (int k = 0; k < kLegTerms; ++k) x[k] = 1.0;
    for (int it = 0; it < 4; ++it) {
        // forward elimination
        double piv = d[0] - sigma;
        wk[0] = piv;
        y[0] = x[0];
        for (int k = 1; k < kLegTerms; ++k) {
            double l = e[k - 1] / wk[k - 1];
            wk[k] = d[k] - sigma - l * e[k - 1];
            y[k] = x[k] - l * y[k - 1];
        }
        x[kLegTerms - 1] = y[kLegTerms - 1] / wk[kLegTerms - 1];
        for (int k = kLegTerms - 2; k >= 0; --k) x[k] = (y[k] - e[k] * x[k + 1]) / wk[k];
        double nrm = 0.0;
        for (int k = 0; k < kLegTerms; ++k) nrm += x[k] * x[k];
        nrm = sqrt(nrm);
        for (int k = 0; k < kLegTerms; ++k) x[k] /= nrm;
    }
    // coefficients of P_{2k}; normalise so that psi(0) = 1
    double p0 = 1.0, val0 = 0.0;
    for (int k = 0; k < kLegTerms; ++k) {
        x[k] *= sqrt((4.0 * k + 1.0) / 2.0);
        val0 += x[k] * p0;
        double n = 2.0 * k;
        p0 = -p0 * (n + 1.0) / (n + 2.0);
    }
    for (int k = 0; k < kLegTerms; ++k) coef[k] = x[k] / val0;
}

__global__ void k_pswf(double c, double *coef) {
    if (threadIdx.x == 0) pswf_coef(c, coef);
}

__device__ double pswf_eval(const double *coef, double eta) {
    // sum_k coef[k] P_{2k}(eta) by the Legendre recurrence
    double pm = 1.0, p = eta;   // P_0, P_1
    double s = coef[0];
    for (int n = 1; n < 2 * kLegTerms - 1; ++n) {
        double pn = ((2.0 * n + 1.0) * eta * p - n * pm) / (n + 1.0);
        pm = p;
        p = pn;
        if (((n + 1) & 1) == 0) s += coef[(n + 1) >> 1] * p;
    }
    return s;
}

// T[j] = psi_0(c, 2 j / M) for j = -M/2 .. M/2 (same normalised abscissae on
// both axes because l_j / (Lx / 2) = 2 j / M)
__global__ void k_taper(const double *coef, int M, int use_ps, double *T) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > M) return;
    int jj = j - M / 2;
    T[j] = use_ps ? pswf_eval(coef, 2.0 * (double)jj / (double)M) : 1.0;
}

__global__ void k_twiddle(int N, double2 *tw) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    double s, c;
    sincospi((double)(2 * r) / (double)N, &s, &c);
    tw[r] = make_double2(c, -s);          // exp(-2 pi i r / N)
}

__device__ __forceinline__ double airy_pow(double x) {
    if (x == 0.0) return 1.0;
    double b = 2.0 * j1(x) / x;
    return b * b;
}

__device__ __forceinline__ double airy_volt(double x) {
    return x == 0.0 ? 1.0 : 2.0 * j1(x) / x;
}

// Mueller kind `kind` of the polarised beam at (l, m): the product of two
// elements of J = [[E_X, d], [d, E_Y]] (kinds E_X^2, E_Y^2, E_X E_Y, E_X d,
// E_Y d, d^2), with elliptical Airy voltage patterns and the four-lobed
// leakage d = kappa (s l)(s m) a(s rho), s = pi D nu / c.
__device__ double pol_beam_kind(int kind, double l, double m, double s, double eta,
                                double kappa) {
    const double lx = l / (1.0 + eta), mx = m / (1.0 - eta);
    const double ly = l / (1.0 - eta), my = m / (1.0 + eta);
    const double ex = airy_volt(s * sqrt(lx * lx + mx * mx));
    const double ey = airy_volt(s * sqrt(ly * ly + my * my));
    const double d = kappa * (s * l) * (s * m) * airy_volt(s * sqrt(l * l + m * m));
    switch (kind) {
        case 0: return ex * ex;
        case 1: return ey * ey;
        case 2: return ex * ey;
        case 3: return ex * d;
        case 4: return ey * d;
        default: return d * d;
    }
}

__global__ void k_screen(CFBuildArgs a, const double *T, double w_k, double nu_fg, double2 *scr) {
    int n1 = a.M + 1;
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n1 * n1) return;
    int i = idx / n1, j = idx - i * n1;
    int ii = i - a.M / 2, jj = j - a.M / 2;
    double l = (double)jj * (a.nx * a.cell_l) / (double)a.M;
    double m = (double)ii * (a.ny * a.cell_m) / (double)a.M;
    double wgt = ((j == 0 || j == a.M) ? 0.5 : 1.0) * ((i == 0 || i == a.M) ? 0.5 : 1.0);
    double re = wgt * T[i] * T[j], im = 0.0;
    if (a.terms & LR_TERM_A) {
        if (a.pol_beam) {
            re *= pol_beam_kind(a.kind, l, m, ((M_PI * a.dish_m) * nu_fg) / kCLight, a.eta,
                                a.kappa);
        } else {
            double rho = sqrt(l * l + m * m);
            re *= airy_pow(((M_PI * a.dish_m) * nu_fg) * rho / kCLight);
        }
    }
    if (a.terms & LR_TERM_W) {
        double r2 = l * l + m * m;
        if (r2 < 1.0) {
            double nm1 = -r2 / (1.0 + sqrt(1.0 - r2));     // sqrt(1 - r^2) - 1
            double s, c;
            sincospi(-2.0 * w_k * nm1, &s, &c);
            im = re * s;
            re = re * c;
        } else {
            re = 0.0;
        }
    }
    scr[idx] = make_double2(re, im);
}

__device__ __forceinline__ int mod_n(int64_t a, int N) {
    int r = (int)(a % N);
    return r < 0 ? r + N : r;
}

// pass 1: A[i][a] = sum_j scr[i][j] exp(-2 pi i n_u (j - M/2) / N), n_u = a - n0
__global__ void k_dft_rows(const double2 *scr, const double2 *tw, int M, int N, int NU,
                           int n0, double2 *A) {
    int n1 = M + 1;
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n1 * NU) return;
    int i = idx / NU, a = idx - i * NU;
    int nu = a - n0;
    double re = 0.0, im = 0.0;
    const double2 *row = scr + (int64_t)i * n1;
    for (int j = 0; j < n1; ++j) {
        double2 t = tw[mod_n((int64_t)nu * (j - M / 2), N)];
        double2 s = row[j];
        re = fma(s.x, t.x, re);
        re = fma(-s.y, t.y, re);
        im = fma(s.x, t.y, im);
        im = fma(s.y, t.x, im);
    }
    A[idx] = make_double2(re, im);
}

// pass 2 + crop: entry (ov, ou, tv, tu) of plane with half-width h.
template <int MODE>   // 0: write f64, 1: write f32, 2: write f64 temp + max
__global__ void k_dft_cols(const double2 *A, const double2 *tw, int M, int N, int NU, int O,
                           int h, double norm, void *out, unsigned long long *maxbits) {
    int S = 2 * h + 1;
    int64_t n_ent = (int64_t)(O + 1) * (O + 1) * S * S;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double mx = 0.0;
    if (idx < n_ent) {
        int tu = (int)(idx % S);
        int64_t r = idx / S;
        int tv = (int)(r % S);
        r /= S;
        int ou = (int)(r % (O + 1));
        int ov = (int)(r / (O + 1));
        int n0 = O / 2 + O * h;
        int nu = (ou - O / 2) - O * (tu - h);
        int nv = (ov - O / 2) - O * (tv - h);
        int au = nu + n0;
        double re = 0.0, im = 0.0;
        for (int i = 0; i <= M; ++i) {
            double2 t = tw[mod_n((int64_t)nv * (i - M / 2), N)];
            double2 s = A[(int64_t)i * NU + au];
            re = fma(s.x, t.x, re);
            re = fma(-s.y, t.y, re);
            im = fma(s.x, t.y, im);
            im = fma(s.y, t.x, im);
        }
        // conj(K) / (M^2 T(0)^2), T(0) = 1
        double vr = re / norm, vi = -im / norm;
        if (MODE == 0) {
            ((double2 *)out)[idx] = make_double2(vr, vi);
        } else if (MODE == 1) {
            ((float2 *)out)[idx] = make_float2((float)vr, (float)vi);
        } else {
            ((double2 *)out)[idx] = make_double2(vr, vi);
            mx = fmax(fabs(vr), fabs(vi));
        }
    }
    if (MODE == 2) {
        // wave max, then one atomic on the bit pattern (monotone for x >= 0)
        for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
        if ((threadIdx.x & 63) == 0)
            atomicMax(maxbits, (unsigned long long)__double_as_longlong(mx));
    }
}

__global__ void k_zero_u64(unsigned long long *p) {
    if (threadIdx.x == 0) *p = 0ull;
}

__global__ void k_plane_exp(const unsigned long long *maxbits, int32_t *exp_out,
                            float *scale_out) {
    if (threadIdx.x != 0) return;
    double mx = __longlong_as_double((long long)*maxbits);
    int e = 0;
    if (mx > 0.0) {
        int ex;
        frexp(mx, &ex);     // mx = f 2^ex, f in [0.5, 1)
        e = -ex;
    }
    *exp_out = e;
    *scale_out = (float)ldexp(1.0, -e);
}

// Round-to-nearest-even of an FP64 value to a binary format with `mbits`
// stored mantissa bits, exponent bias `bias`, minimum normal exponent
// `emin` (unbiased); returns the bit pattern.  Finite inputs of magnitude
// below the format's overflow threshold only.
__device__ __forceinline__ uint32_t round_small_float(double x, int mbits, int bias, int emin) {
    uint32_t sign = signbit(x) ? 1u : 0u;
    double a = fabs(x);
    uint32_t bits;
    if (a == 0.0) {
        bits = 0;
    } else {
        int ex;
        double f = frexp(a, &ex);           // a = f 2^ex, f in [0.5, 1)
        int e = ex - 1;                     // a = (2f) 2^e, 2f in [1, 2)
        if (e >= emin) {
            double q = rint(ldexp(f, mbits + 1));       // in [2^mbits, 2^(mbits+1)]
            uint64_t m = (uint64_t)q;
            if (m == (1ull << (mbits + 1))) { m >>= 1; e += 1; }
            bits = ((uint32_t)(e + bias) << mbits) | (uint32_t)(m - (1ull << mbits));
        } else {
            // subnormal: units of 2^(emin - mbits); may round up to the
            // smallest normal, whose encoding follows on naturally
            bits = (uint32_t)rint(ldexp(a, mbits - emin));
        }
    }
    int tot = 1 + mbits + (mbits == 10 ? 5 : 8);
    return (sign << (tot - 1)) | bits;
}

template <int BF16>
__global__ void k_convert16(const double2 *src, int64_t n, const int32_t *exp_in,
                            uint32_t *dst) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int e = *exp_in;
    double2 v = src[i];
    double re = ldexp(v.x, e), im = ldexp(v.y, e);
    uint32_t a, b;
    if (BF16) {
        a = round_small_float(re, 7, 127, -126);
        b = round_small_float(im, 7, 127, -126);
    } else {
        a = round_small_float(re, 10, 15, -14);
        b = round_small_float(im, 10, 15, -14);
    }
    dst[i] = a | (b << 16);
}

__global__ void k_unit_scale(int32_t *exps, float *scales, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        exps[i] = 0;
        scales[i] = 1.0f;
    }
}

size_t cf_work_bytes(int32_t M, int32_t O, int32_t h_max) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    int64_t N = (int64_t)O * M;
    int64_t S = 2 * h_max + 1;
    int64_t NU = O * S + 1;
    size_t b = 0;
    b += al(sizeof(double) * kLegTerms);
    b += al(sizeof(double) * (M + 1));
    b += al(sizeof(double2) * N);
    b += al(sizeof(double2) * (M + 1) * (M + 1));
    b += al(sizeof(double2) * (M + 1) * NU);
    b += al(sizeof(double2) * (O + 1) * (O + 1) * S * S);
    b += al(64);
    return b;
}

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// The PS term's taper at n image pixels, psi_0(c, 2 (i - n/2) / n) (the
// screen's taper sampled at the pixels; 1 without a PS term).  One
// workgroup: the first thread finds the Legendre coefficients.
__global__ void k_ps_taper(double c, int use_ps, int32_t n, double *out) {
    __shared__ double coef[kLegTerms];
    if (use_ps && threadIdx.x == 0) pswf_coef(c, coef);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        out[i] = use_ps ? pswf_eval(coef, 2.0 * (double)(i - n / 2) / (double)n) : 1.0;
}

hipError_t launch_ps_taper(double c, int use_ps, int32_t n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_ps_taper, dim3(1), dim3(256), 0, s, c, use_ps, n, out);
    return hipGetLastError();
}

// Weight image of A-projection: every pixel of every (plane, pol) gets
// sum_fg w[fg] B_fg(rho)^2 / sum_fg w[fg], B_fg the Airy power pattern of
// the table's A term at the group's frequency (x = fscale[fg] rho).
struct PBArgs {
    double fscale[128];     // pi D nu_fg / c of every group
    int32_t nx, ny, n_fg, use_a;
    double cell_l, cell_m;
    int64_t n_planes;
};

__global__ void k_pb_image(PBArgs a, const double *w, double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)a.nx * a.ny;
    if (i >= per * a.n_planes) return;
    const int64_t pl = i / per;
    const int64_t r = i - pl * per;
    const int iy = (int)(r / a.nx), ix = (int)(r - (int64_t)iy * a.nx);
    const double l = (double)(ix - a.nx / 2) * a.cell_l, m = (double)(iy - a.ny / 2) * a.cell_m;
    const double rho = sqrt(l * l + m * m);
    const double *wp = w + pl * a.n_fg;
    double num = 0.0, den = 0.0;
    for (int g = 0; g < a.n_fg; ++g) {
        const double b = a.use_a ? airy_pow(a.fscale[g] * rho) : 1.0;
        num += wp[g] * (b * b);
        den += wp[g];
    }
    out[i] = den > 0.0 ? num / den : 0.0;
}

hipError_t launch_pb_image(const lr_cf *cf, const double *w, double *out, hipStream_t s) {
    const lr_grid_spec &g = cf->grid;
    PBArgs a;
    a.n_fg = cf->spec.n_fg;
    for (int k = 0; k < 128; ++k)
        a.fscale[k] = k < a.n_fg ? M_PI * cf->spec.dish_m * cf->fg_hz[k] / kCLight : 0.0;
    a.nx = g.nx;
    a.ny = g.ny;
    a.use_a = (cf->spec.terms & LR_TERM_A) ? 1 : 0;
    a.cell_l = g.cell_l;
    a.cell_m = g.cell_m;
    a.n_planes = (int64_t)g.nplane * g.npol;
    const int64_t n = (int64_t)g.nx * g.ny * a.n_planes;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pb_image, dim3(nblk(n, 256)), dim3(256), 0, s, a, w, out);
    return hipGetLastError();
}

hipError_t launch_cf_build(const lr_cf *cf, const CFBuildArgs &a0, void *work, hipStream_t s) {
    CFBuildArgs a = a0;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const lr_cf_spec &sp = cf->spec;
    int M = a.M, O = a.O;
    int N = O * M;
    int hmax = 0;
    for (int v : cf->h) hmax = v > hmax ? v : hmax;
    int64_t Smax = 2 * hmax + 1;
    int NUmax = (int)(O * Smax + 1);
    char *w = (char *)work;
    double *coef = (double *)w;           w += al(sizeof(double) * kLegTerms);
    double *T = (double *)w;              w += al(sizeof(double) * (M + 1));
    double2 *tw = (double2 *)w;           w += al(sizeof(double2) * N);
    double2 *scr = (double2 *)w;          w += al(sizeof(double2) * (M + 1) * (M + 1));
    double2 *A = (double2 *)w;            w += al(sizeof(double2) * (M + 1) * NUmax);
    double2 *plane = (double2 *)w;        w += al(sizeof(double2) * (O + 1) * (O + 1) * Smax * Smax);
    unsigned long long *maxbits = (unsigned long long *)w;

    int use_ps = (a.terms & LR_TERM_PS) ? 1 : 0;
    if (use_ps) hipLaunchKernelGGL(k_pswf, dim3(1), dim3(64), 0, s, a.c_ps, coef);
    hipLaunchKernelGGL(k_taper, dim3(nblk(M + 1, 256)), dim3(256), 0, s, coef, M, use_ps, T);
    hipLaunchKernelGGL(k_twiddle, dim3(nblk(N, 256)), dim3(256), 0, s, N, tw);
    int n_planes = sp.n_fg * sp.n_w;
    int st = sp.storage;
    if (st == LR_F64 || st == LR_F32)
        hipLaunchKernelGGL(k_unit_scale, dim3(nblk(n_planes * cf->n_kind, 256)), dim3(256), 0,
                           s, cf->d_exp, cf->d_scale, n_planes * cf->n_kind);
    double norm = (double)M * (double)M;
    for (int kind = 0; kind < cf->n_kind; ++kind) {
        a.kind = kind;
        for (int g = 0; g < sp.n_fg; ++g) {
            for (int k = 0; k < sp.n_w; ++k) {
                double w_k = sp.n_w > 1 ? ((double)k * sp.w_max) / (double)(sp.n_w - 1) : 0.0;
                int h = cf->h[k];
                int S = 2 * h + 1;
                int NU = O * S + 1;
                int n0 = O / 2 + O * h;
                hipLaunchKernelGGL(k_screen, dim3(nblk((int64_t)(M + 1) * (M + 1), 256)),
                                   dim3(256), 0, s, a, T, w_k, cf->fg_hz[g], scr);
                hipLaunchKernelGGL(k_dft_rows, dim3(nblk((int64_t)(M + 1) * NU, 256)), dim3(256),
                                   0, s, scr, tw, M, N, NU, n0, A);
                // plane index of the scale arrays (kind-major) and the plane's
                // place in the table (each kind laid out as the scalar table)
                int pi = kind * n_planes + g * sp.n_w + k;
                int64_t n_ent = (int64_t)(O + 1) * (O + 1) * S * S;
                char *dst = (char *)cf->d_table +
                            (kind * cf->kind_elems + cf->plane_off[g * sp.n_w + k]) * cf->elem_bytes;
                if (st == LR_F64) {
                    hipLaunchKernelGGL(k_dft_cols<0>, dim3(nblk(n_ent, 256)), dim3(256), 0, s, A,
                                       tw, M, N, NU, O, h, norm, (void *)dst, maxbits);
                } else if (st == LR_F32) {
                    hipLaunchKernelGGL(k_dft_cols<1>, dim3(nblk(n_ent, 256)), dim3(256), 0, s, A,
                                       tw, M, N, NU, O, h, norm, (void *)dst, maxbits);
                } else {
                    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, maxbits);
                    hipLaunchKernelGGL(k_dft_cols<2>, dim3(nblk(n_ent, 256)), dim3(256), 0, s, A,
                                       tw, M, N, NU, O, h, norm, (void *)plane, maxbits);
                    hipLaunchKernelGGL(k_plane_exp, dim3(1), dim3(64), 0, s, maxbits,
                                       cf->d_exp + pi, cf->d_scale + pi);
                    if (st == LR_F32_CF16)
                        hipLaunchKernelGGL(k_convert16<0>, dim3(nblk(n_ent, 256)), dim3(256), 0, s,
                                           plane, n_ent, cf->d_exp + pi, (uint32_t *)dst);
                    else
                        hipLaunchKernelGGL(k_convert16<1>, dim3(nblk(n_ent, 256)), dim3(256), 0, s,
                                           plane, n_ent, cf->d_exp + pi, (uint32_t *)dst);
                }
            }
        }
    }
    return hipGetLastError();
}

}  // namespace lr
