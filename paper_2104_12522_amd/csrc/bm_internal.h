// Internal declarations and device helpers of libbartmi (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include "bartmi.h"

namespace bm {

// ---- physical constants, CGS -----------------------------------------------------------
constexpr double kBoltz = 1.380649e-16;        // erg / K
constexpr double kAmu = 1.66053906660e-24;     // g
constexpr double kLight = 2.99792458e10;       // cm / s
constexpr double kC2 = 1.4387769;              // h c / k_B, cm K
constexpr double kGrav = 6.67430e-8;           // cm^3 g^-1 s^-2
constexpr double kBar = 1.0e6;                 // dyn / cm^2
constexpr double kAtmBar = 1.01325;            // bar
constexpr double kTRef = 296.0;                // K
constexpr double kRJup = 7.1492e9;             // cm (IAU equatorial)
constexpr double kEulerGamma = 0.57721566490153286061;

constexpr int kWave = 64;

#define BM_CHECK_HIP(expr)                                   \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return BM_EHIP;                \
    } while (0)

// ---- E2 exponential integral -------------------------------------------------------------
// x <= 2.5: E2 = e^-x - x E1, E1 by its power series (Abramowitz & Stegun 5.1.11),
//           E1(x) = -gamma - ln x - sum_{k>=1} (-x)^k / (k k!), 24 terms;
// x >  2.5: E2 by the even continued fraction (A&S 5.1.22),
//           E2 = e^-x / (x + 2 - 1*2 / (x + 4 - 2*3 / (x + 6 - ...))),
//           through its convergents P_n / Q_n (three-term recurrence, one division) at
//           a fixed depth of 39, at least what 8 + 75/x (about 1e-14 relative) asks for at the
//           smallest x = 2.5: every larger x has converged further, and a loop of the
//           same length on every lane needs no per-lane exit tests.
struct E1SeriesCoef {
    double c[24];  // c[k-1] = (-1)^k / (k k!)
    constexpr E1SeriesCoef() : c() {
        double fact = 1.0;
        for (int k = 1; k <= 24; ++k) {
            fact *= k;
            c[k - 1] = ((k & 1) ? -1.0 : 1.0) / (k * fact);
        }
    }
};

// ex = exp(-x) supplied by the caller (it is shared with the profile's other term)
__host__ __device__ inline double expint_e2_ex(double x, double ex) {
    if (x <= 0.0) return 1.0;
    if (x <= 2.5) {
        // the polynomial sum_{k<24} c_k x^k as its even and odd parts in x^2, two
        // independent Horner chains of 12 steps
        constexpr E1SeriesCoef cs;
        const double x2 = x * x;
        double se = cs.c[22], so = cs.c[23];
        for (int k = 20; k >= 0; k -= 2) {
            se = fma(se, x2, cs.c[k]);
            so = fma(so, x2, cs.c[k + 1]);
        }
        const double s = x * fma(so, x, se);  // sum_{k>=1} c_k x^k
        double e1 = -kEulerGamma - log(x) - s;
        return ex - x * e1;
    }
    // denominator b_1 - a_2/(b_2 - a_3/(...)), b_m = x + 2m, a_m = (m-1) m, with the
    // recurrence P_m = b_m P_{m-1} - a_m P_{m-2} (same for Q) software-pipelined: the term
    // a_{m+1} P_{m-1} of the next step is formed alongside step m, so one multiply-add per
    // step lies on the dependent chain
    constexpr int kDepth = 39;  // 38 steps (an even count for the unrolled loop)
    double p1 = x + 2.0, q1 = 1.0;  // P_1, Q_1
    double tp = -2.0, tq = 0.0;     // -a_2 P_0, -a_2 Q_0 (P_0 = 1, Q_0 = 0)
    double bm = x + 2.0;            // b_{m-1}; b_m = b_{m-1} + 2
    double an = 2.0;                // a_m; a_{m+1} = a_m + 2 m (exact in double)
#pragma unroll 2
    for (int m = 2; m <= kDepth; ++m) {
        bm += 2.0;
        an += 2.0 * m;
        const double p2 = fma(bm, p1, tp), q2 = fma(bm, q1, tq);
        tp = -an * p1;
        tq = -an * q1;
        p1 = p2;
        q1 = q2;
    }
    return ex * q1 / p1;
}

__host__ __device__ inline double expint_e2(double x) { return expint_e2_ex(x, exp(-x)); }

__host__ __device__ inline double pow10_(double x) { return exp2(x * 3.32192809488736234787); }

// H2 Rayleigh-scattering cross section (cm^2) at wavenumber nu (cm^-1): the Dalgarno &
// Williams (1962) series in inverse powers of the wavelength in Angstrom (terms in
// lambda^-4, lambda^-6, lambda^-8), evaluated in Horner form in lambda^-2.
__host__ __device__ inline double rayleigh_h2_xsec(double nu) {
    const double inv_lam = nu * 1.0e-8;  // 1 / (lambda in Angstrom)
    const double q = inv_lam * inv_lam;
    return q * q * (8.14e-13 + q * (1.28e-6 + q * 1.61));
}

// ---- Line et al. (2013) five-parameter temperature profile ------------------------------
// Per-sample constants of the profile, evaluated once per sample.
struct Line2013Consts {
    double kappa_over_g;   // kappa / g_nom
    double g1, g2;         // gamma_1, gamma_2
    double alpha;
    double tirr4, tint4;   // T_irr^4, T_int^4
};

__host__ __device__ inline Line2013Consts line2013_consts(const double* tp, const bm_planet& pl) {
    Line2013Consts c;
    c.kappa_over_g = pow10_(tp[0]) / pl.g_nom;
    c.g1 = pow10_(tp[1]);
    c.g2 = pow10_(tp[2]);
    c.alpha = tp[3];
    const double tirr = tp[4] * sqrt(pl.rstar_cm / (2.0 * pl.a_cm)) * pl.tstar;
    c.tirr4 = (tirr * tirr) * (tirr * tirr);
    c.tint4 = (pl.tint * pl.tint) * (pl.tint * pl.tint);
    return c;
}

// xi(gamma, tau) = 2/3 + 2/(3 gamma) [1 + (gamma tau / 2 - 1) e^{-gamma tau}]
//                  + (2 gamma / 3)(1 - tau^2 / 2) E2(gamma tau)
__host__ __device__ inline double line2013_xi(double gamma, double tau) {
    const double gt = gamma * tau;
    const double ex = exp(-gt);
    return 2.0 / 3.0 + 2.0 / (3.0 * gamma) * (1.0 + (gt * 0.5 - 1.0) * ex) +
           2.0 * gamma / 3.0 * (1.0 - tau * tau * 0.5) * expint_e2_ex(gt, ex);
}

// T^4 = 3/4 T_int^4 (2/3 + tau) + 3/4 T_irr^4 [(1 - alpha) xi(gamma_1) + alpha xi(gamma_2)],
// tau = kappa p / g
__host__ __device__ inline double line2013_tau(double p_bar, const Line2013Consts& c) {
    return c.kappa_over_g * (p_bar * kBar);
}
__host__ __device__ inline double line2013_temperature_xi(double tau, double xi1, double xi2,
                                                          const Line2013Consts& c) {
    const double t4 = 0.75 * c.tint4 * (2.0 / 3.0 + tau) + 0.75 * c.tirr4 * (1.0 - c.alpha) * xi1 +
                      0.75 * c.tirr4 * c.alpha * xi2;
    return sqrt(sqrt(t4));
}
__host__ __device__ inline double line2013_temperature_c(double p_bar, const Line2013Consts& c) {
    const double tau = line2013_tau(p_bar, c);
    return line2013_temperature_xi(tau, line2013_xi(c.g1, tau), line2013_xi(c.g2, tau), c);
}

__host__ __device__ inline double line2013_temperature(double p_bar, const double* tp, const bm_planet& pl) {
    return line2013_temperature_c(p_bar, line2013_consts(tp, pl));
}

// ---- linear-in-T interpolation bracket --------------------------------------------------
// k = largest index with grid[k] <= t, clamped to [0, n-2]; w = (t - g_k)/(g_{k+1} - g_k)
// clamped to [0, 1]; returns true when t lies outside [grid[0], grid[n-1]].
__host__ __device__ inline bool interp_bracket(const double* grid, int n, double t, int* k_out,
                                               double* w_out) {
    int k = 0;
#pragma unroll 8
    for (int i = 1; i < n; ++i)
        if (grid[i] <= t) k = i;
    if (k > n - 2) k = n - 2;
    double w = (t - grid[k]) / (grid[k + 1] - grid[k]);
    bool clamped = !(grid[0] <= t && t <= grid[n - 1]);
    w = w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
    if (!(w == w)) w = 0.0;  // NaN temperature: flagged elsewhere
    *k_out = k;
    *w_out = w;
    return clamped;
}

// Half-chord length from the tangent point at radius rj to the sphere of radius rl.
__host__ __device__ inline double half_chord(double rl, double rj) {
    return sqrt((rl - rj) * (rl + rj));
}

template <typename T>
struct DType;
template <>
struct DType<float> {
    static constexpr int code = BM_F32;
};
template <>
struct DType<double> {
    static constexpr int code = BM_F64;
};

// Absorbed fraction 1 - exp(-t) of a chord of optical depth t >= 0 (the integrand of the
// transit-depth integral, Sec. 6.1). FP32: the Taylor polynomial of degree 7 below t = 0.35
// (truncation under 2e-8 relative) and 1 - 2^(-t log2 e) from 0.35 up, where the result is
// at least 0.29 and the subtraction loses nothing; both are evaluated and one is selected,
// so that the chord loops carry no divergent branch. Within 3e-7 relative of the exact
// value (a correctly rounded result is within 6e-8), at a third of expm1f's instructions.
// FP64: -expm1(-t).
__device__ __forceinline__ float dev_absorbed(float t) {
    float p = 1.f / 5040.f;
    p = fmaf(p, t, -1.f / 720.f);
    p = fmaf(p, t, 1.f / 120.f);
    p = fmaf(p, t, -1.f / 24.f);
    p = fmaf(p, t, 1.f / 6.f);
    p = fmaf(p, t, -0.5f);
    p = fmaf(p, t, 1.f);
    const float small = p * t;
    const float large = 1.f - __builtin_amdgcn_exp2f(-1.44269504f * t);
    return t < 0.35f ? small : large;
}
__device__ __forceinline__ double dev_absorbed(double t) { return -expm1(-t); }

}  // namespace bm
