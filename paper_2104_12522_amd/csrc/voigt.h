// Faddeeva function and Voigt helpers shared by the opacity builds (internal).
//
// Re w(z), double precision:
//   |z| >= 8   Laplace continued fraction of w(z), evaluated through its convergents
//              P_m / Q_m (one division), 4-10 levels depending on |z|;
//   |z| <  8   Weideman (1994) rational expansion with N = 40 terms, whose coefficients
//              are computed on the host from the FFT (here a direct cosine sum) of
//              (L^2 + t^2) exp(-t^2) sampled at t = L tan(theta / 2).
#pragma once

#include <vector>

#include "bm_internal.h"

namespace bm {

constexpr int kWeidemanN = 40;

struct WeidemanCoef {
    double L;
    double a[kWeidemanN];  // a_1 .. a_N
};

inline WeidemanCoef weideman_coefficients() {
    WeidemanCoef c{};
    const int N = kWeidemanN;
    const int M = 2 * N;
    const double L = sqrt(N / sqrt(2.0));
    c.L = L;
    const double pi = 3.14159265358979323846;
    std::vector<double> g(2 * M);
    for (int m = 0; m < 2 * M; ++m) {
        if (m == M) {
            g[m] = 0.0;  // theta = pi, t = infinity
            continue;
        }
        const double t = L * tan(0.5 * pi * m / M);
        g[m] = exp(-t * t) * (L * L + t * t);
    }
    for (int n = 1; n <= N; ++n) {
        double s = 0.0;
        for (int m = 0; m < 2 * M; ++m) s += g[m] * cos(pi * (double)n * m / M);
        c.a[n - 1] = s / (2.0 * M);
    }
    return c;
}

// Re w(x + i y) far from the origin (|z| >= 8): the Laplace continued fraction of w(z),
// 1/(z - (1/2)/(z - (2/2)/(z - ...))), through its convergents P_m / Q_m with
// h_m = z h_{m-1} - ((m-1)/2) h_{m-2} (P_0 = 0, P_1 = 1; Q_0 = 1, Q_1 = z), N levels; then
// w = (i / sqrt(pi)) P / Q, Re w = -Im(P / Q) / sqrt(pi). N is a compile-time depth, so the
// recurrence unrolls into straight-line code with no register rotation.
template <int N>
__device__ __forceinline__ double faddeeva_re_cf(double x, double y) {
    double pr0 = 0.0, pi0 = 0.0, pr1 = 1.0, pi1 = 0.0;
    double qr0 = 1.0, qi0 = 0.0, qr1 = x, qi1 = y;
#pragma unroll
    for (int m = 2; m <= N + 1; ++m) {
        const double am = -0.5 * (m - 1);
        const double prn = x * pr1 - y * pi1 + am * pr0;
        const double pin = x * pi1 + y * pr1 + am * pi0;
        const double qrn = x * qr1 - y * qi1 + am * qr0;
        const double qin = x * qi1 + y * qr1 + am * qi0;
        pr0 = pr1; pi0 = pi1; pr1 = prn; pi1 = pin;
        qr0 = qr1; qi0 = qi1; qr1 = qrn; qi1 = qin;
    }
    const double den = qr1 * qr1 + qi1 * qi1;
    const double im_ratio = (pi1 * qr1 - pr1 * qi1) / den;
    return -im_ratio * 0.56418958354775628695;  // 1/sqrt(pi)
}

// Re w(x + i y), y > 0.
__device__ __forceinline__ double faddeeva_re(double x, double y, const WeidemanCoef& wc) {
    x = fabs(x);
    const double r2 = x * x + y * y;
    // depth by |z|: 4 levels for |z| >= 40 (every evaluation of strongly pressure-broadened
    // lines), 6 from 15, 8 from 10, 10 from 8. The depth is taken uniform over the wave's
    // active lanes that use the fraction: the deepest any of them needs. A deeper
    // convergent is as accurate (within 3.1e-14 relative of Re w over |z| >= 8, against
    // scipy's wofz), and lanes spread over several |z| bands then run one unrolled
    // recurrence instead of each band's in turn.
    if (r2 >= 64.0) {
        if (!__ballot(r2 < 1600.0)) return faddeeva_re_cf<4>(x, y);  // the common case first
        if (__ballot(r2 < 100.0)) return faddeeva_re_cf<10>(x, y);
        if (__ballot(r2 < 225.0)) return faddeeva_re_cf<8>(x, y);
        return faddeeva_re_cf<6>(x, y);
    }
    // Weideman: Z = (L + iz)/(L - iz), w = (2 p(Z) / (L - iz) + 1/sqrt(pi)) / (L - iz)
    const double L = wc.L;
    const double dr = L + y, di = -x;            // L - iz
    const double dd = 1.0 / (dr * dr + di * di);
    const double ir = dr * dd, ii = -di * dd;    // 1 / (L - iz)
    const double nr = L - y, ni = x;             // L + iz
    const double zr = nr * ir - ni * ii, zi = nr * ii + ni * ir;
    double pr = wc.a[kWeidemanN - 1], pim = 0.0;
#pragma unroll
    for (int n = kWeidemanN - 2; n >= 0; --n) {
        const double tr = pr * zr - pim * zi + wc.a[n];
        const double ti = pr * zi + pim * zr;
        pr = tr;
        pim = ti;
    }
    // t = 2 p / (L - iz) + 1/sqrt(pi)
    const double tr = 2.0 * (pr * ir - pim * ii) + 0.56418958354775628695;
    const double ti = 2.0 * (pr * ii + pim * ir);
    return tr * ir - ti * ii;
}

// Re w(x + i y) far from the origin in single precision, for single-precision tables: the
// same N-level truncation of the Laplace continued fraction, evaluated from the innermost
// level outwards, t = z, t <- z - (k/2)/t for k = N .. 1, w = (i / sqrt(pi)) / t, so
// Re w = Im t / (sqrt(pi) |t|^2). Every quantity stays of the order of |z| (no convergent
// growth, so no overflow at any |z|); each level is one reciprocal and four fused
// multiply-adds, with a relative rounding of a few units of the last place.
template <int N>
__device__ __forceinline__ float faddeeva_re_cf_f32(float x, float y) {
    float tr = x, ti = y;
#pragma unroll
    for (int k = N; k >= 1; --k) {
        const float c = (0.5f * (float)k) * __builtin_amdgcn_rcpf(fmaf(tr, tr, ti * ti));
        tr = fmaf(-c, tr, x);
        ti = fmaf(c, ti, y);
    }
    return ti * __builtin_amdgcn_rcpf(fmaf(tr, tr, ti * ti)) * 0.56418958f;  // 1/sqrt(pi)
}

// Re w for single-precision tables: the continued fraction in single precision where
// |z| >= 8 (every point of pressure-broadened lines' windows), Weideman's expansion in
// double inside |z| < 8 (line cores, where its terms cancel)
__device__ __forceinline__ double faddeeva_re_f32wings(double x, double y, const WeidemanCoef& wc) {
    x = fabs(x);
    const double r2 = x * x + y * y;
    if (r2 >= 64.0) {
        const float xf = (float)x, yf = (float)y;
        if (!__ballot(r2 < 1600.0)) return faddeeva_re_cf_f32<4>(xf, yf);
        if (__ballot(r2 < 100.0)) return faddeeva_re_cf_f32<10>(xf, yf);
        if (__ballot(r2 < 225.0)) return faddeeva_re_cf_f32<8>(xf, yf);
        return faddeeva_re_cf_f32<6>(xf, yf);
    }
    return faddeeva_re(x, y, wc);
}

__device__ __forceinline__ double voigt_hwhm(double sig, double gam) {
    return 0.5346 * gam + sqrt(0.2166 * gam * gam + 2.0 * 0.69314718055994530942 * sig * sig);
}

// the coefficients, computed once per process
inline const WeidemanCoef& weideman() {
    static const WeidemanCoef c = weideman_coefficients();
    return c;
}

// Voigt profile V(x; sig, gam) = Re w((x + i gam) / (sig sqrt 2)) / (sig sqrt(2 pi))
__device__ __forceinline__ double voigt_profile(double x, double sig, double gam, const WeidemanCoef& wc) {
    const double inv = 1.0 / (sig * 1.41421356237309504880);
    return faddeeva_re(x * inv, gam * inv, wc) / (sig * 2.50662827463100050242);
}

}  // namespace bm
