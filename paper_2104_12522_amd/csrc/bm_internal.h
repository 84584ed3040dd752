// Internal declarations and device helpers of libbartmi (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include "../../include/bartmi.h"

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
// E1 by its power series for x <= 1 (Abramowitz & Stegun 5.1.11) and E_n by the even
// continued fraction for x > 1 (A&S 5.1.22), evaluated backwards at fixed depth.
__host__ __device__ inline double expint_e2(double x) {
    if (x <= 0.0) return 1.0;
    if (x <= 1.0) {
        // E1(x) = -gamma - ln x - sum_{k>=1} (-x)^k / (k k!)
        double term = 1.0, sum = 0.0;
        for (int k = 1; k <= 24; ++k) {
            term *= -x / k;
            sum += term / k;
        }
        double e1 = -kEulerGamma - log(x) - sum;
        return exp(-x) - x * e1;  // E2 = e^-x - x E1
    }
    // E_2(x) = e^-x / (x + 2 - 1*2 / (x + 4 - 2*3 / (x + 6 - ...)))
    const int depth = 60;
    double t = x + 2.0 + 2.0 * depth;
    for (int m = depth; m >= 1; --m) {
        t = x + 2.0 + 2.0 * (m - 1) - (double)m * (double)(m + 1) / t;
    }
    return exp(-x) / t;
}

// ---- Line et al. (2013) five-parameter temperature profile ------------------------------
__host__ __device__ inline double line2013_xi(double gamma, double tau) {
    double gt = gamma * tau;
    return 2.0 / 3.0 + 2.0 / (3.0 * gamma) * (1.0 + (gt * 0.5 - 1.0) * exp(-gt)) +
           2.0 * gamma / 3.0 * (1.0 - tau * tau * 0.5) * expint_e2(gt);
}

__host__ __device__ inline double line2013_temperature(double p_bar, const double* tp,
                                                       const bm_planet& pl) {
    double kappa = pow(10.0, tp[0]);
    double g1 = pow(10.0, tp[1]);
    double g2 = pow(10.0, tp[2]);
    double alpha = tp[3], beta = tp[4];
    double tau = kappa * (p_bar * kBar) / pl.g_nom;
    double tirr = beta * sqrt(pl.rstar_cm / (2.0 * pl.a_cm)) * pl.tstar;
    double tirr4 = tirr * tirr * tirr * tirr;
    double tint4 = pl.tint * pl.tint * pl.tint * pl.tint;
    double t4 = 0.75 * tint4 * (2.0 / 3.0 + tau) +
                0.75 * tirr4 * (1.0 - alpha) * line2013_xi(g1, tau) +
                0.75 * tirr4 * alpha * line2013_xi(g2, tau);
    return sqrt(sqrt(t4));
}

// ---- linear-in-T interpolation bracket --------------------------------------------------
// k = largest index with grid[k] <= t, clamped to [0, n-2]; w = (t - g_k)/(g_{k+1} - g_k)
// clamped to [0, 1]; returns true when t lies outside [grid[0], grid[n-1]].
__host__ __device__ inline bool interp_bracket(const double* grid, int n, double t, int* k_out,
                                               double* w_out) {
    int k = 0;
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

__device__ inline float dev_expm1(float x) { return expm1f(x); }
__device__ inline double dev_expm1(double x) { return expm1(x); }

}  // namespace bm
