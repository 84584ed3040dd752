// Secondary path: line-by-line opacity table (Sec. 3 and Sec. 4, first pass; Sec. 6.1.1,
// Voigt profile Eqs. 4-11; Sec. 4, point sampling at the output wavenumbers).
//
// Kernels k_opacity_gather and k_opacity_narrow: one workgroup owns 256 consecutive output
// wavenumbers of one (T, p) cell. The lines are sorted by centre, so the lines that can
// reach the tile form one index range, found by binary search with the widest possible
// window of the cell. The range is staged through LDS 256 lines at a time (per-line
// strength, Doppler and Lorentz widths and window computed once per workgroup). Each cell
// is built by one of the two kernels, chosen by its widest window: wavenumber-major (every
// lane sums the profiles of the staged lines whose window contains its wavenumber) or, for
// windows of a few grid points, line-major (threads evaluate each line's window points,
// then every lane sums its own). Both sum in double, in line order, with no atomics: each
// output element is written once, so results are deterministic. The Faddeeva function is
// in voigt.h.
#include <algorithm>
#include <type_traits>

#include "voigt.h"

namespace bm {

constexpr int kOpThreads = 256;

struct LineArrays {
    const double* nu0;
    const double* s296;
    const double* gamma296;
    const double* elow;
    const double* mass;
    int64_t n;
};

// (T, p) cells of the table, passed by value: cell c = it * n_p + ip.
struct CellGrid {
    double temp[BM_MAX_TEMPS];
    double p_bar[BM_MAX_LAYERS];
    int n_p;
};

// Line-list extremes in the caller's workspace, in two stages: up to kExtBlocks workgroups
// each reduce a grid-strided share of the lines into the partials ws[kExtFinal + 4 b ..],
// one workgroup then reduces those into ws[0..4): max gamma296, max nu0 / sqrt(mass) (the
// widest-window inputs), min gamma296, min nu0 / sqrt(mass). Maxima and minima are exact in
// any order. With no lines the final stage writes max 0 and min +inf.
constexpr int kExtBlocks = 256;
constexpr int kExtFinal = 4;
constexpr size_t kExtWorkspaceBytes = sizeof(double) * (kExtFinal + 4 * kExtBlocks);
struct Ext4 {
    double gmax, dmax, gmin, dmin;
};
__device__ __forceinline__ Ext4 block_ext4(Ext4 v, Ext4* s) {
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            Ext4& a = s[threadIdx.x];
            const Ext4 b = s[threadIdx.x + off];
            a.gmax = fmax(a.gmax, b.gmax);
            a.dmax = fmax(a.dmax, b.dmax);
            a.gmin = fmin(a.gmin, b.gmin);
            a.dmin = fmin(a.dmin, b.dmin);
        }
        __syncthreads();
    }
    return s[0];
}

__global__ void __launch_bounds__(256) k_line_extremes(LineArrays ln, double* ws) {
    __shared__ Ext4 s[256];
    Ext4 v{0.0, 0.0, __builtin_huge_val(), __builtin_huge_val()};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ln.n; i += (int64_t)gridDim.x * blockDim.x) {
        const double g = ln.gamma296[i];
        const double d = ln.nu0[i] / sqrt(ln.mass[i]);
        v.gmax = fmax(v.gmax, g);
        v.dmax = fmax(v.dmax, d);
        v.gmin = fmin(v.gmin, g);
        v.dmin = fmin(v.dmin, d);
    }
    v = block_ext4(v, s);
    if (threadIdx.x == 0) {
        double* o = ws + kExtFinal + 4 * blockIdx.x;
        o[0] = v.gmax;
        o[1] = v.dmax;
        o[2] = v.gmin;
        o[3] = v.dmin;
    }
}

__global__ void __launch_bounds__(256) k_line_extremes_final(double* ws, int n_blocks) {
    __shared__ Ext4 s[256];
    Ext4 v{0.0, 0.0, __builtin_huge_val(), __builtin_huge_val()};
    for (int b = threadIdx.x; b < n_blocks; b += blockDim.x) {
        const double* o = ws + kExtFinal + 4 * b;
        v.gmax = fmax(v.gmax, o[0]);
        v.dmax = fmax(v.dmax, o[1]);
        v.gmin = fmin(v.gmin, o[2]);
        v.dmin = fmin(v.dmin, o[3]);
    }
    v = block_ext4(v, s);
    if (threadIdx.x == 0) {
        ws[0] = v.gmax;
        ws[1] = v.dmax;
        ws[2] = v.gmin;
        ws[3] = v.dmin;
    }
}

// Range of the Doppler sigma and Lorentz gamma that the lines take over the cells with
// temperatures in [t_lo, t_hi] and pressures in [p_lo, p_hi] (bar), from the extremes:
// out = {sigma_min, sigma_max, gamma_min, gamma_max}
__global__ void k_width_range(const double* __restrict__ ext, double t_lo, double t_hi, double p_lo,
                              double p_hi, double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    out[0] = ext[3] / kLight * sqrt(kBoltz * t_lo / kAmu);
    out[1] = ext[1] / kLight * sqrt(kBoltz * t_hi / kAmu);
    out[2] = ext[2] * (p_lo / kAtmBar) * sqrt(kTRef / t_hi);
    out[3] = ext[0] * (p_hi / kAtmBar) * sqrt(kTRef / t_lo);
}

// the cell's widest window plus one grid step: every line's window is at most wmax - dnu
// wide (the Doppler and Lorentz widths of the widest line bound every line's; the factor
// covers their rounding)
__device__ __forceinline__ double cell_wmax(const double* __restrict__ extremes, double T_, double pfac,
                                            double cutoff, double dnu) {
    const double gmax = extremes[0] * pfac;
    const double smax = extremes[1] / kLight * sqrt(kBoltz * T_ / kAmu);
    return cutoff * voigt_hwhm(smax, gmax) * (1.0 + 1e-12) + dnu;
}

// Cells of narrow lines take the line-major kernel: every window, widened by two grid points
// on each side for rounding, spans at most kNarrowPts points.
constexpr int kNarrowPts = 48;
constexpr int kNarrowLines = 64;  // lines evaluated per pass, four threads each
__device__ __forceinline__ bool narrow_cell(double wmax, double dnu) {
    return 2.0 * wmax / dnu + 3.0 <= (double)kNarrowPts;
}

// first line with nu0 >= lo_v and first line with nu0 > hi_v (centres sorted ascending)
__device__ inline void line_range(const LineArrays& ln, double lo_v, double hi_v, int64_t* range) {
    int64_t a = 0, b = ln.n;
    while (a < b) {
        int64_t mid = (a + b) >> 1;
        if (ln.nu0[mid] < lo_v) a = mid + 1; else b = mid;
    }
    range[0] = a;
    b = ln.n;
    while (a < b) {
        int64_t mid = (a + b) >> 1;
        if (ln.nu0[mid] <= hi_v) a = mid + 1; else b = mid;
    }
    range[1] = a;
}

// Re w at the table's precision: single-precision tables take the single-precision far-wing
// evaluation (each term then carries a relative rounding of ~1e-6, the sum stays in double)
template <typename T>
__device__ __forceinline__ double faddeeva_t(double x, double y, const WeidemanCoef& wc) {
    if constexpr (sizeof(T) == 4) return faddeeva_re_f32wings(x, y, wc);
    return faddeeva_re(x, y, wc);
}

// Lines staged in LDS: centre, window half-width, S(T) / (sigma sqrt(2 pi)), 1 / (sigma sqrt 2)
// and the Faddeeva argument's imaginary part y = gamma / (sigma sqrt 2).
struct StagedLines {
    double nu0[kOpThreads], half[kOpThreads], amp[kOpThreads], inv[kOpThreads], y[kOpThreads];
};

// line i at temperature T_ into slot t (Sec. 3: strength at T, Doppler and Lorentz widths)
__device__ __forceinline__ void stage_line(const LineArrays& ln, int64_t i, int t, double T_, double pfac,
                                           double cutoff, double qratio, StagedLines& sl) {
    const double boltz_ref = 1.0 / kTRef;
    const double nu0 = ln.nu0[i];
    const double el = ln.elow[i];
    const double s_t = ln.s296[i] * qratio * exp(-kC2 * el / T_) / exp(-kC2 * el * boltz_ref) *
                       ((1.0 - exp(-kC2 * nu0 / T_)) / (1.0 - exp(-kC2 * nu0 * boltz_ref)));
    const double sig = nu0 / kLight * sqrt(kBoltz * T_ / (ln.mass[i] * kAmu));
    const double gam = ln.gamma296[i] * pfac;
    const double inv = 1.0 / (sig * 1.41421356237309504880);
    sl.nu0[t] = nu0;
    sl.half[t] = cutoff * voigt_hwhm(sig, gam);
    sl.amp[t] = s_t / (sig * 2.50662827463100050242);  // sigma sqrt(2 pi)
    sl.inv[t] = inv;
    sl.y[t] = gam * inv;
}

// Wavenumber-major build (cells of wide lines): every lane sums, in line order, the profiles
// of the staged lines whose window contains its wavenumber.
template <typename T>
__global__ void __launch_bounds__(kOpThreads)
    k_opacity_gather(LineArrays ln, CellGrid cg, double nu_start, double dnu, int n_nu, double cutoff,
                     const double* __restrict__ extremes, WeidemanCoef wc, T* __restrict__ out) {
    __shared__ StagedLines sl;
    __shared__ int64_t range[2];
    const int cell = blockIdx.y;
    const double T_ = cg.temp[cell / cg.n_p];
    const double p = cg.p_bar[cell % cg.n_p];
    const int k = blockIdx.x * kOpThreads + threadIdx.x;
    const double nu = nu_start + dnu * (double)k;
    const double t_lo = nu_start + dnu * (double)(blockIdx.x * kOpThreads);
    const double t_hi = nu_start + dnu * (double)min(blockIdx.x * kOpThreads + kOpThreads - 1, n_nu - 1);

    const double pfac = (p / kAtmBar) * sqrt(kTRef / T_);
    const double wmax = cell_wmax(extremes, T_, pfac, cutoff, dnu);
    if (narrow_cell(wmax, dnu)) return;  // the line-major kernel builds this cell
    if (threadIdx.x == 0) line_range(ln, t_lo - wmax, t_hi + wmax, range);
    __syncthreads();
    const int64_t first = range[0], last = range[1];
    const double qratio = pow(kTRef / T_, 1.5);
    double acc = 0.0;
    for (int64_t c0 = first; c0 < last; c0 += kOpThreads) {
        const int64_t i = c0 + threadIdx.x;
        if (i < last) stage_line(ln, i, threadIdx.x, T_, pfac, cutoff, qratio, sl);
        __syncthreads();
        const int cnt = (int)min((int64_t)kOpThreads, last - c0);
        if (k < n_nu) {
            for (int q = 0; q < cnt; ++q) {
                const double d = nu - sl.nu0[q];
                if (fabs(d) <= sl.half[q]) acc += sl.amp[q] * faddeeva_t<T>(d * sl.inv[q], sl.y[q], wc);
            }
        }
        __syncthreads();
    }
    if (k < n_nu) out[(size_t)cell * n_nu + k] = (T)acc;
}

// Line-major build (cells of narrow lines, whose windows span a few grid points: in the
// wavenumber-major loop most of a wave would idle through each line's profile). Per pass
// of 64 staged lines, four threads per line evaluate the profile at the line's window
// points inside the tile into LDS, marking each evaluated point; then every lane adds, in
// line order, the marked values at its own wavenumber. Same terms and order as the
// wavenumber-major kernel; each value is the same double, kept as a float for a float
// table.
template <typename T>
__global__ void __launch_bounds__(kOpThreads)
    k_opacity_narrow(LineArrays ln, CellGrid cg, double nu_start, double dnu, int n_nu, double cutoff,
                     const double* __restrict__ extremes, WeidemanCoef wc, T* __restrict__ out) {
    __shared__ StagedLines sl;
    // profile values, point j of the line's span: float for a float table (each term then
    // carries a relative error of 6e-8, the table's own resolution; the sum stays in
    // double), which halves the buffer and raises the workgroups per CU from 4 to 6
    using FVal = typename std::conditional<sizeof(T) == 4, float, double>::type;
    __shared__ FVal s_f[kNarrowLines][kNarrowPts];
    __shared__ unsigned long long s_mask[kNarrowLines][4];  // bit j of mask[j % 4]: value j was evaluated
    __shared__ int s_k0[kNarrowLines], s_n[kNarrowLines];   // first grid point and length of the span
    __shared__ int64_t range[2];
    static_assert(kNarrowPts <= 64 && kNarrowLines * 4 == kOpThreads, "pass layout");
    const int cell = blockIdx.y;
    const double T_ = cg.temp[cell / cg.n_p];
    const double p = cg.p_bar[cell % cg.n_p];
    const int tile0 = blockIdx.x * kOpThreads;
    const int tile1 = min(tile0 + kOpThreads - 1, n_nu - 1);
    const int k = tile0 + threadIdx.x;
    const double nu = nu_start + dnu * (double)k;
    const double t_lo = nu_start + dnu * (double)(blockIdx.x * kOpThreads);
    const double t_hi = nu_start + dnu * (double)min(blockIdx.x * kOpThreads + kOpThreads - 1, n_nu - 1);

    const double pfac = (p / kAtmBar) * sqrt(kTRef / T_);
    const double wmax = cell_wmax(extremes, T_, pfac, cutoff, dnu);
    if (!narrow_cell(wmax, dnu)) return;  // the wavenumber-major kernel builds this cell
    if (threadIdx.x == 0) line_range(ln, t_lo - wmax, t_hi + wmax, range);
    __syncthreads();
    const int64_t first = range[0], last = range[1];
    const double qratio = pow(kTRef / T_, 1.5);
    const int ql = threadIdx.x >> 2, r = threadIdx.x & 3;
    double acc = 0.0;
    for (int64_t c0 = first; c0 < last; c0 += kOpThreads) {
        const int64_t i = c0 + threadIdx.x;
        if (i < last) stage_line(ln, i, threadIdx.x, T_, pfac, cutoff, qratio, sl);
        __syncthreads();
        const int cnt = (int)min((int64_t)kOpThreads, last - c0);
        for (int sub = 0; sub < cnt; sub += kNarrowLines) {
            const int q = sub + ql;
            unsigned long long mask = 0;
            if (q < cnt) {
                // grid points that can lie in the window, one point of margin on each side
                // (kb - ka + 1 <= 2 half / dnu + 5 <= 2 wmax / dnu + 3 <= kNarrowPts),
                // clipped to the tile
                const double nu0 = sl.nu0[q], half = sl.half[q];
                const int ka = max((int)floor((nu0 - half - nu_start) / dnu) - 1, tile0);
                const int kb = min((int)ceil((nu0 + half - nu_start) / dnu) + 1, tile1);
                const int n = min(kb - ka + 1, kNarrowPts);
                if (r == 0) {
                    s_k0[ql] = ka;
                    s_n[ql] = n;
                }
                for (int j = r; j < n; j += 4) {
                    const double d = (nu_start + dnu * (double)(ka + j)) - nu0;
                    if (fabs(d) <= half) {
                        s_f[ql][j] = (FVal)faddeeva_t<T>(d * sl.inv[q], sl.y[q], wc);
                        mask |= 1ull << j;
                    }
                }
            }
            s_mask[ql][r] = mask;
            __syncthreads();
            if (k < n_nu) {
                const int qn = min(kNarrowLines, cnt - sub);
                for (int l = 0; l < qn; ++l) {
                    const int j = k - s_k0[l];
                    if (j >= 0 && j < s_n[l] && ((s_mask[l][j & 3] >> j) & 1ull))
                        acc += sl.amp[sub + l] * (double)s_f[l][j];
                }
            }
            __syncthreads();
        }
    }
    if (k < n_nu) out[(size_t)cell * n_nu + k] = (T)acc;
}

__global__ void k_voigt(const double* __restrict__ x, int64_t n, double sig, double gam, WeidemanCoef wc,
                        double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double inv = 1.0 / (sig * 1.41421356237309504880);
    out[i] = faddeeva_re(x[i] * inv, gam * inv, wc) / (sig * 2.50662827463100050242);
}

}  // namespace bm

using namespace bm;

extern "C" int bm_voigt(const double* x, int64_t n, double sigma, double gamma, double* out, void* stream) {
    if (!x || !out) return BM_EINVAL;
    if (n < 0) return BM_ESHAPE;
    if (!(sigma > 0.0) || !(gamma > 0.0)) return BM_EINVAL;
    if (n == 0) return BM_OK;
    const int threads = 256;
    hipLaunchKernelGGL(k_voigt, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0,
                       (hipStream_t)stream, x, n, sigma, gamma, weideman(), out);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

static void launch_line_extremes(const LineArrays& ln, double* ws, hipStream_t st) {
    const int nb = (int)std::min<int64_t>(kExtBlocks, (ln.n + 255) / 256);
    if (nb > 0) hipLaunchKernelGGL(k_line_extremes, dim3(nb), dim3(256), 0, st, ln, ws);
    hipLaunchKernelGGL(k_line_extremes_final, dim3(1), dim3(256), 0, st, ws, nb);
}

extern "C" size_t bm_opacity_build_workspace(int64_t n_lines) {
    if (n_lines < 0) return 0;
    return kExtWorkspaceBytes;
}

extern "C" int bm_line_width_range(const double* nu0, const double* gamma296, const double* mass_amu,
                                   int64_t n_lines, const double* temp, int n_temp, const double* p_bar,
                                   int n_p, double* range_out, void* workspace, size_t workspace_bytes,
                                   void* stream) {
    if (!nu0 || !gamma296 || !mass_amu || !temp || !p_bar || !range_out || !workspace) return BM_EINVAL;
    if (n_lines < 1 || n_temp < 1 || n_p < 1) return BM_ESHAPE;
    if (workspace_bytes < kExtWorkspaceBytes) return BM_ENOSPACE;
    double t_lo = temp[0], t_hi = temp[0], p_lo = p_bar[0], p_hi = p_bar[0];
    for (int i = 0; i < n_temp; ++i) {
        if (!(temp[i] > 0.0)) return BM_EINVAL;
        t_lo = std::min(t_lo, temp[i]);
        t_hi = std::max(t_hi, temp[i]);
    }
    for (int i = 0; i < n_p; ++i) {
        if (!(p_bar[i] > 0.0)) return BM_EINVAL;
        p_lo = std::min(p_lo, p_bar[i]);
        p_hi = std::max(p_hi, p_bar[i]);
    }
    hipStream_t st = (hipStream_t)stream;
    double* ws = (double*)workspace;
    LineArrays ln{nu0, nullptr, gamma296, nullptr, mass_amu, n_lines};
    launch_line_extremes(ln, ws, st);
    BM_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_width_range, dim3(1), dim3(64), 0, st, ws, t_lo, t_hi, p_lo, p_hi, range_out);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

extern "C" int bm_opacity_table_build(const double* nu0, const double* s296, const double* gamma296,
                                      const double* elow, const double* mass_amu, int64_t n_lines,
                                      const double* temp, int n_temp, const double* p_bar, int n_p,
                                      double nu_start, double dnu, int n_nu, double cutoff_hwhm, int dtype,
                                      void* sigma_out, void* workspace, size_t workspace_bytes,
                                      void* stream) {
    if (!temp || !p_bar || !sigma_out || !workspace) return BM_EINVAL;
    if (n_lines > 0 && (!nu0 || !s296 || !gamma296 || !elow || !mass_amu)) return BM_EINVAL;
    if (n_lines < 0 || n_temp < 1 || n_temp > BM_MAX_TEMPS || n_p < 1 || n_p > BM_MAX_LAYERS || n_nu < 1)
        return BM_ESHAPE;
    if (!(dnu > 0.0) || !(cutoff_hwhm > 0.0)) return BM_EINVAL;
    if (dtype != BM_F32 && dtype != BM_F64) return BM_EINVAL;
    if (workspace_bytes < kExtWorkspaceBytes) return BM_ENOSPACE;
    CellGrid cg{};
    for (int i = 0; i < n_temp; ++i) {
        if (!(temp[i] > 0.0)) return BM_EINVAL;
        cg.temp[i] = temp[i];
    }
    for (int i = 0; i < n_p; ++i) {
        if (!(p_bar[i] > 0.0)) return BM_EINVAL;
        cg.p_bar[i] = p_bar[i];
    }
    cg.n_p = n_p;
    hipStream_t st = (hipStream_t)stream;
    // the widest-window inputs, written on every call (with no lines: zeros, and every
    // cell's line range is empty)
    double* d_ext = (double*)workspace;
    LineArrays ln{nu0, s296, gamma296, elow, mass_amu, n_lines};
    launch_line_extremes(ln, d_ext, st);
    BM_CHECK_HIP(hipGetLastError());
    dim3 grid((n_nu + kOpThreads - 1) / kOpThreads, n_temp * n_p);
    // every cell is built by exactly one of the two kernels (the other's workgroups exit)
    if (dtype == BM_F32) {
        hipLaunchKernelGGL(k_opacity_gather<float>, grid, dim3(kOpThreads), 0, st, ln, cg, nu_start, dnu, n_nu,
                           cutoff_hwhm, d_ext, weideman(), (float*)sigma_out);
        BM_CHECK_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_opacity_narrow<float>, grid, dim3(kOpThreads), 0, st, ln, cg, nu_start, dnu, n_nu,
                           cutoff_hwhm, d_ext, weideman(), (float*)sigma_out);
    } else {
        hipLaunchKernelGGL(k_opacity_gather<double>, grid, dim3(kOpThreads), 0, st, ln, cg, nu_start, dnu,
                           n_nu, cutoff_hwhm, d_ext, weideman(), (double*)sigma_out);
        BM_CHECK_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_opacity_narrow<double>, grid, dim3(kOpThreads), 0, st, ln, cg, nu_start, dnu,
                           n_nu, cutoff_hwhm, d_ext, weideman(), (double*)sigma_out);
    }
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}
