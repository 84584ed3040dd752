// Secondary path: line-by-line opacity table (Sec. 3 and Sec. 4, first pass; Sec. 6.1.1,
// Voigt profile Eqs. 4-11; Sec. 4, point sampling at the output wavenumbers).
//
// Kernel k_opacity_gather: one workgroup owns 256 consecutive output wavenumbers of one
// (T, p) cell. The lines are sorted by centre, so the lines that can reach the tile form
// one index range, found by binary search with the widest possible window of the cell.
// The range is staged through LDS 256 lines at a time (per-line strength, Doppler and
// Lorentz widths and window computed once per workgroup), and every lane sums the
// profiles of the staged lines whose window contains its wavenumber, in double, in line
// order. No atomics: each output element is written once, so results are deterministic.
// The Faddeeva function is in voigt.h.
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

// widest window inputs over all lines: [0] max gamma296, [1] max nu0 / sqrt(mass)
__global__ void k_line_extremes(LineArrays ln, double* out) {
    __shared__ double s0[256], s1[256];
    double g = 0.0, d = 0.0;
    for (int64_t i = threadIdx.x; i < ln.n; i += blockDim.x) {
        g = fmax(g, ln.gamma296[i]);
        d = fmax(d, ln.nu0[i] / sqrt(ln.mass[i]));
    }
    s0[threadIdx.x] = g;
    s1[threadIdx.x] = d;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            s0[threadIdx.x] = fmax(s0[threadIdx.x], s0[threadIdx.x + off]);
            s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s0[0];
        out[1] = s1[0];
    }
}

template <typename T>
__global__ void __launch_bounds__(kOpThreads)
    k_opacity_gather(LineArrays ln, CellGrid cg, double nu_start, double dnu, int n_nu, double cutoff,
                     const double* __restrict__ extremes, WeidemanCoef wc, T* __restrict__ out) {
    __shared__ double s_nu0[kOpThreads], s_half[kOpThreads], s_amp[kOpThreads], s_inv[kOpThreads],
        s_y[kOpThreads];
    __shared__ int64_t range[2];
    const int cell = blockIdx.y;
    const double T_ = cg.temp[cell / cg.n_p];
    const double p = cg.p_bar[cell % cg.n_p];
    const int k = blockIdx.x * kOpThreads + threadIdx.x;
    const double nu = nu_start + dnu * (double)k;
    const double t_lo = nu_start + dnu * (double)(blockIdx.x * kOpThreads);
    const double t_hi = nu_start + dnu * (double)min(blockIdx.x * kOpThreads + kOpThreads - 1, n_nu - 1);

    const double pfac = (p / kAtmBar) * sqrt(kTRef / T_);
    if (threadIdx.x == 0) {
        const double gmax = extremes[0] * pfac;
        const double smax = extremes[1] / kLight * sqrt(kBoltz * T_ / kAmu);
        const double wmax = cutoff * voigt_hwhm(smax, gmax) * (1.0 + 1e-12) + dnu;
        // first line with nu0 >= t_lo - wmax, first line with nu0 > t_hi + wmax
        const double lo_v = t_lo - wmax, hi_v = t_hi + wmax;
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
    __syncthreads();
    const int64_t first = range[0], last = range[1];
    const double boltz_ref = 1.0 / kTRef;
    const double qratio = pow(kTRef / T_, 1.5);
    double acc = 0.0;
    for (int64_t c0 = first; c0 < last; c0 += kOpThreads) {
        const int64_t i = c0 + threadIdx.x;
        if (i < last) {
            const double nu0 = ln.nu0[i];
            const double el = ln.elow[i];
            const double s_t = ln.s296[i] * qratio * exp(-kC2 * el / T_) / exp(-kC2 * el * boltz_ref) *
                               ((1.0 - exp(-kC2 * nu0 / T_)) / (1.0 - exp(-kC2 * nu0 * boltz_ref)));
            const double sig = nu0 / kLight * sqrt(kBoltz * T_ / (ln.mass[i] * kAmu));
            const double gam = ln.gamma296[i] * pfac;
            const double inv = 1.0 / (sig * 1.41421356237309504880);
            s_nu0[threadIdx.x] = nu0;
            s_half[threadIdx.x] = cutoff * voigt_hwhm(sig, gam);
            s_amp[threadIdx.x] = s_t / (sig * 2.50662827463100050242);  // sigma sqrt(2 pi)
            s_inv[threadIdx.x] = inv;
            s_y[threadIdx.x] = gam * inv;
        }
        __syncthreads();
        const int cnt = (int)min((int64_t)kOpThreads, last - c0);
        if (k < n_nu) {
            for (int q = 0; q < cnt; ++q) {
                const double d = nu - s_nu0[q];
                if (fabs(d) <= s_half[q]) acc += s_amp[q] * faddeeva_re(d * s_inv[q], s_y[q], wc);
            }
        }
        __syncthreads();
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

// The widest-window inputs (two doubles) live in a 256-byte buffer per device, allocated
// on the first call on that device and held until the process ends.
static double* extremes_buffer() {
    static double* per_device[64] = {nullptr};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    if (!per_device[dev]) {
        void* p = nullptr;
        if (hipMalloc(&p, 256) != hipSuccess) return nullptr;
        per_device[dev] = (double*)p;
    }
    return per_device[dev];
}

extern "C" int bm_opacity_table_build(const double* nu0, const double* s296, const double* gamma296,
                                      const double* elow, const double* mass_amu, int64_t n_lines,
                                      const double* temp, int n_temp, const double* p_bar, int n_p,
                                      double nu_start, double dnu, int n_nu, double cutoff_hwhm, int dtype,
                                      void* sigma_out, void* stream) {
    if (!temp || !p_bar || !sigma_out) return BM_EINVAL;
    if (n_lines > 0 && (!nu0 || !s296 || !gamma296 || !elow || !mass_amu)) return BM_EINVAL;
    if (n_lines < 0 || n_temp < 1 || n_temp > BM_MAX_TEMPS || n_p < 1 || n_p > BM_MAX_LAYERS || n_nu < 1)
        return BM_ESHAPE;
    if (!(dnu > 0.0) || !(cutoff_hwhm > 0.0)) return BM_EINVAL;
    if (dtype != BM_F32 && dtype != BM_F64) return BM_EINVAL;
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
    double* d_ext = extremes_buffer();
    if (!d_ext) return BM_EHIP;
    LineArrays ln{nu0, s296, gamma296, elow, mass_amu, n_lines};
    if (n_lines > 0) hipLaunchKernelGGL(k_line_extremes, dim3(1), dim3(256), 0, st, ln, d_ext);
    BM_CHECK_HIP(hipGetLastError());
    dim3 grid((n_nu + kOpThreads - 1) / kOpThreads, n_temp * n_p);
    if (dtype == BM_F32)
        hipLaunchKernelGGL(k_opacity_gather<float>, grid, dim3(kOpThreads), 0, st, ln, cg, nu_start, dnu, n_nu,
                           cutoff_hwhm, d_ext, weideman(), (float*)sigma_out);
    else
        hipLaunchKernelGGL(k_opacity_gather<double>, grid, dim3(kOpThreads), 0, st, ln, cg, nu_start, dnu,
                           n_nu, cutoff_hwhm, d_ext, weideman(), (double*)sigma_out);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}
