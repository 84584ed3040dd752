// Secondary path, profile-table mode: the opacity build as the paper describes it (Sec. 4
// items 4-6 and the paragraph after them; Sec. 6.1.1 for the 60 x 60 profile grid).
//
// Profile table. Profile (i, j) is V(t delta; sigma_i, gamma_j) for t = -T..T fine steps,
// delta = dnu / O (O samples per output interval, so the samples align with the output
// grid), T = floor(cutoff HWHM_ij / delta), stored in single precision. A line whose
// centre is s fine steps from nu_start (s = rint((nu0 - nu_start) / delta)) reaches the
// output points k with u = k O - s + T in [0, 2T]; all such points share the residue
// u mod O, so each profile is stored residue-major, row rho = u mod O holding
// u = rho, rho + O, ..., and the points of one line read consecutive floats.
// Layout of the table buffer: a header (int64 ext[n], rows[n], off[n + 1]; double
// sigma nodes, gamma nodes and their geometric midpoints), then the float rows from
// byte data_off; off[] counts floats.
//
// Build (k_opacity_profiles): one workgroup per (T, p) cell and 256 output points, as in
// the direct mode. Lines are staged 256 at a time; each gets its strength S(T), widths,
// nearest nodes (the midpoints decide), shift and the strength test against the
// strongest line at that temperature. Runs of consecutive lines with the same profile and
// shift are merged by a segmented scan of their strengths (item 5: one broadening per
// run), then every lane adds S P(u) for its point, in line order, in double.
#include "voigt.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

// The integer decisions (extents, nearest nodes, shifts) come from arithmetic written
// operation by operation, on the host and on the device alike.
#pragma clang fp contract(off)

namespace bm {

constexpr int kPfThreads = 256;
constexpr int kPfNodesMax = 256;
constexpr int kPfStatBlocks = 128;  // partial maxima per temperature in the statistics pass

struct ProfileLayout {
    int n_sigma = 0, n_gamma = 0, n = 0;
    int64_t oversample = 0;
    double delta = 0.0, dnu = 0.0;
    std::vector<int64_t> ext, rows, off;
    std::vector<double> snode, gnode, smid, gmid;
    size_t hdr_bytes = 0, data_off = 0, total_bytes = 0;
};

struct ProfileView {
    const int64_t* ext;
    const int64_t* rows;
    const int64_t* off;
    const double* snode;
    const double* gnode;
    const double* smid;
    const double* gmid;
    const float* data;
    int n_sigma, n_gamma, n;
    int64_t oversample;
    double delta;
};

static size_t pf_align(size_t x, size_t a) { return (x + a - 1) / a * a; }

static double table_hwhm(double sig, double gam) {
    return 0.5346 * gam + std::sqrt(0.2166 * gam * gam + 1.3862943611198906 * sig * sig);
}

static int profile_layout(const bm_voigt_grid* g, ProfileLayout& L) {
    if (!g || !g->sigma_nodes || !g->gamma_nodes) return BM_EINVAL;
    if (g->n_sigma < 1 || g->n_sigma > kPfNodesMax || g->n_gamma < 1 || g->n_gamma > kPfNodesMax) return BM_ESHAPE;
    if (g->oversample < 1 || g->oversample > 65536) return BM_ESHAPE;
    if (!(g->dnu > 0.0) || !std::isfinite(g->dnu) || !(g->cutoff_hwhm > 0.0) || !std::isfinite(g->cutoff_hwhm))
        return BM_EINVAL;
    for (int i = 0; i < g->n_sigma; ++i)
        if (!(g->sigma_nodes[i] > 0.0) || !std::isfinite(g->sigma_nodes[i]) ||
            (i > 0 && !(g->sigma_nodes[i] > g->sigma_nodes[i - 1])))
            return BM_EINVAL;
    for (int j = 0; j < g->n_gamma; ++j)
        if (!(g->gamma_nodes[j] > 0.0) || !std::isfinite(g->gamma_nodes[j]) ||
            (j > 0 && !(g->gamma_nodes[j] > g->gamma_nodes[j - 1])))
            return BM_EINVAL;
    L.n_sigma = g->n_sigma;
    L.n_gamma = g->n_gamma;
    L.n = g->n_sigma * g->n_gamma;
    L.oversample = g->oversample;
    L.dnu = g->dnu;
    L.delta = g->dnu / (double)g->oversample;
    L.snode.assign(g->sigma_nodes, g->sigma_nodes + g->n_sigma);
    L.gnode.assign(g->gamma_nodes, g->gamma_nodes + g->n_gamma);
    L.smid.assign(std::max(1, L.n_sigma - 1), 0.0);
    L.gmid.assign(std::max(1, L.n_gamma - 1), 0.0);
    for (int i = 0; i + 1 < L.n_sigma; ++i) L.smid[i] = std::sqrt(L.snode[i] * L.snode[i + 1]);
    for (int j = 0; j + 1 < L.n_gamma; ++j) L.gmid[j] = std::sqrt(L.gnode[j] * L.gnode[j + 1]);
    L.ext.resize(L.n);
    L.rows.resize(L.n);
    L.off.resize(L.n + 1);
    L.off[0] = 0;
    const double max_floats = 4.0e11;
    for (int i = 0; i < L.n_sigma; ++i)
        for (int j = 0; j < L.n_gamma; ++j) {
            const int p = i * L.n_gamma + j;
            const double t = std::floor(g->cutoff_hwhm * table_hwhm(L.snode[i], L.gnode[j]) / L.delta);
            if (!(t >= 0.0) || t > max_floats) return BM_ESHAPE;
            L.ext[p] = (int64_t)t;
            L.rows[p] = (2 * L.ext[p]) / L.oversample + 1;
            L.off[p + 1] = L.off[p] + L.oversample * L.rows[p];
            if ((double)L.off[p + 1] > max_floats) return BM_ESHAPE;
        }
    L.hdr_bytes = sizeof(int64_t) * (3 * (size_t)L.n + 1) +
                  sizeof(double) * (L.snode.size() + L.gnode.size() + L.smid.size() + L.gmid.size());
    L.data_off = pf_align(L.hdr_bytes, 256);
    L.total_bytes = L.data_off + sizeof(float) * (size_t)L.off[L.n];
    return BM_OK;
}

// the header in one host buffer, in device order
static std::vector<char> layout_header(const ProfileLayout& L) {
    std::vector<char> h(L.hdr_bytes);
    char* p = h.data();
    auto put = [&](const void* src, size_t bytes) {
        std::memcpy(p, src, bytes);
        p += bytes;
    };
    put(L.ext.data(), sizeof(int64_t) * L.n);
    put(L.rows.data(), sizeof(int64_t) * L.n);
    put(L.off.data(), sizeof(int64_t) * (L.n + 1));
    put(L.snode.data(), sizeof(double) * L.snode.size());
    put(L.gnode.data(), sizeof(double) * L.gnode.size());
    put(L.smid.data(), sizeof(double) * L.smid.size());
    put(L.gmid.data(), sizeof(double) * L.gmid.size());
    return h;
}

static ProfileView layout_view(const ProfileLayout& L, const void* table) {
    const char* b = static_cast<const char*>(table);
    ProfileView v{};
    v.ext = reinterpret_cast<const int64_t*>(b);
    v.rows = v.ext + L.n;
    v.off = v.rows + L.n;
    v.snode = reinterpret_cast<const double*>(v.off + L.n + 1);
    v.gnode = v.snode + L.snode.size();
    v.smid = v.gnode + L.gnode.size();
    v.gmid = v.smid + L.smid.size();
    v.data = reinterpret_cast<const float*>(b + L.data_off);
    v.n_sigma = L.n_sigma;
    v.n_gamma = L.n_gamma;
    v.n = L.n;
    v.oversample = L.oversample;
    v.delta = L.delta;
    return v;
}

// profile values, residue-major: entry e of profile p is row rho = r / rows, column
// c = r % rows (r = e - off[p]), i.e. fine offset u = c O + rho, t = u - T
__global__ void k_profile_fill(ProfileView pv, int64_t total, WeidemanCoef wc, float* __restrict__ data) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = pv.n;  // off[lo] <= e < off[hi]
        while (hi - lo > 1) {
            const int m = (lo + hi) >> 1;
            if (pv.off[m] <= e) lo = m; else hi = m;
        }
        const int64_t r = e - pv.off[lo], nr = pv.rows[lo], T = pv.ext[lo];
        const int64_t rho = r / nr, c = r - rho * nr;
        const int64_t u = c * pv.oversample + rho;
        float v = 0.0f;
        if (u <= 2 * T) {
            const double x = (double)(u - T) * pv.delta;
            v = (float)voigt_profile(x, pv.snode[lo / pv.n_gamma], pv.gnode[lo % pv.n_gamma], wc);
        }
        data[e] = v;
    }
}

struct PfLines {
    const double* nu0;
    const double* s296;
    const double* gamma296;
    const double* elow;
    const double* mass;
    int64_t n;
};

struct PfCells {
    double temp[BM_MAX_TEMPS];
    double p_bar[BM_MAX_LAYERS];
    int n_t, n_p;
};

// S(T) = S_296 (296/T)^1.5 exp(-c2 E''/T) / exp(-c2 E''/296) (1 - exp(-c2 nu0/T)) /
// (1 - exp(-c2 nu0/296))
__device__ __forceinline__ double pf_strength(double s296, double nu0, double el, double T, double qratio) {
    const double boltz = exp(-kC2 * el / T) / exp(-kC2 * el / kTRef);
    const double stim = (1.0 - exp(-kC2 * nu0 / T)) / (1.0 - exp(-kC2 * nu0 / kTRef));
    return s296 * qratio * boltz * stim;
}

// number of midpoints <= x: the node nearest to x in ratio
__device__ __forceinline__ int pf_nearest(const double* mid, int n_nodes, double x) {
    int lo = 0, hi = n_nodes - 1;
    while (lo < hi) {
        const int m = (lo + hi) >> 1;
        if (mid[m] <= x) lo = m + 1; else hi = m;
    }
    return lo;
}

// Workspace (doubles): part_s[n_t][kPfStatBlocks], part_g[kPfStatBlocks],
// part_d[kPfStatBlocks], smax[n_t], extremes[2] (max gamma296, max nu0 / sqrt(mass)).
static size_t pf_workspace_doubles(int n_t) { return (size_t)n_t * kPfStatBlocks + 2 * kPfStatBlocks + n_t + 2; }

__global__ void __launch_bounds__(kPfThreads) k_line_stats(PfLines ln, PfCells cg, double* __restrict__ ws) {
    __shared__ double r0[kPfThreads], r1[kPfThreads], r2[kPfThreads];
    const int it = blockIdx.y, b = blockIdx.x;
    const double T = cg.temp[it];
    const double qratio = pow(kTRef / T, 1.5);
    double ms = 0.0, mg = 0.0, md = 0.0;
    for (int64_t i = (int64_t)b * kPfThreads + threadIdx.x; i < ln.n; i += (int64_t)kPfStatBlocks * kPfThreads) {
        ms = fmax(ms, pf_strength(ln.s296[i], ln.nu0[i], ln.elow[i], T, qratio));
        if (it == 0) {
            mg = fmax(mg, ln.gamma296[i]);
            md = fmax(md, ln.nu0[i] / sqrt(ln.mass[i]));
        }
    }
    r0[threadIdx.x] = ms;
    r1[threadIdx.x] = mg;
    r2[threadIdx.x] = md;
    __syncthreads();
    for (int o = kPfThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            r0[threadIdx.x] = fmax(r0[threadIdx.x], r0[threadIdx.x + o]);
            r1[threadIdx.x] = fmax(r1[threadIdx.x], r1[threadIdx.x + o]);
            r2[threadIdx.x] = fmax(r2[threadIdx.x], r2[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ws[(size_t)it * kPfStatBlocks + b] = r0[0];
        if (it == 0) {
            ws[(size_t)cg.n_t * kPfStatBlocks + b] = r1[0];
            ws[(size_t)cg.n_t * kPfStatBlocks + kPfStatBlocks + b] = r2[0];
        }
    }
}

__global__ void k_line_stats_final(int n_t, double* __restrict__ ws) {
    const int t = threadIdx.x;
    double* smax = ws + (size_t)n_t * kPfStatBlocks + 2 * kPfStatBlocks;
    if (t < n_t + 2) {
        const double* src = (t < n_t) ? ws + (size_t)t * kPfStatBlocks
                                      : ws + (size_t)n_t * kPfStatBlocks + (size_t)(t - n_t) * kPfStatBlocks;
        double m = 0.0;
        for (int b = 0; b < kPfStatBlocks; ++b) m = fmax(m, src[b]);
        smax[t] = m;  // smax[n_t], smax[n_t + 1] are the two extremes
    }
}

template <typename T>
__global__ void __launch_bounds__(kPfThreads)
    k_opacity_profiles(PfLines ln, PfCells cg, double nu_start, double dnu, int n_nu, ProfileView pv,
                       double strength_cutoff, const double* __restrict__ ws, T* __restrict__ out) {
    __shared__ int64_t s_shift[kPfThreads], s_u0[kPfThreads], s_2t[kPfThreads], s_base[kPfThreads];
    __shared__ int s_pid[kPfThreads];
    __shared__ double s_S[kPfThreads];
    __shared__ int s_flag[kPfThreads];
    __shared__ int64_t range[2];
    const int cell = blockIdx.y;
    const int it = cell / cg.n_p;
    const double Tc = cg.temp[it];
    const double p = cg.p_bar[cell % cg.n_p];
    const int j = threadIdx.x;
    const int64_t k0 = (int64_t)blockIdx.x * kPfThreads;
    const int64_t k = k0 + j;
    const int64_t O = pv.oversample;
    const double* smax = ws + (size_t)cg.n_t * kPfStatBlocks + 2 * kPfStatBlocks;
    const double pf = p / kAtmBar;
    const double sq = sqrt(kTRef / Tc);
    if (j == 0) {
        // the widest profile any line of this cell can take: nodes nearest the largest
        // widths, one node further for safety (extents grow with both widths)
        const double gmax = (smax[cg.n_t] * pf) * sq;
        const double dmax = (smax[cg.n_t + 1] / kLight) * sqrt((kBoltz * Tc) / kAmu);
        const int is = min(pf_nearest(pv.smid, pv.n_sigma, dmax) + 1, pv.n_sigma - 1);
        const int ig = min(pf_nearest(pv.gmid, pv.n_gamma, gmax) + 1, pv.n_gamma - 1);
        const double w = (double)(pv.ext[is * pv.n_gamma + ig] + 2) * pv.delta + dnu;
        const double t_lo = nu_start + dnu * (double)k0;
        const double t_hi = nu_start + dnu * (double)min(k0 + kPfThreads - 1, (int64_t)n_nu - 1);
        const double lo_v = t_lo - w, hi_v = t_hi + w;
        int64_t a = 0, b = ln.n;
        while (a < b) {
            const int64_t mid = (a + b) >> 1;
            if (ln.nu0[mid] < lo_v) a = mid + 1; else b = mid;
        }
        range[0] = a;
        b = ln.n;
        while (a < b) {
            const int64_t mid = (a + b) >> 1;
            if (ln.nu0[mid] <= hi_v) a = mid + 1; else b = mid;
        }
        range[1] = a;
    }
    __syncthreads();
    const int64_t first = range[0], last = range[1];
    const double thr = strength_cutoff * smax[it];
    const double qratio = pow(kTRef / Tc, 1.5);
    double acc = 0.0;
    for (int64_t c0 = first; c0 < last; c0 += kPfThreads) {
        const int cnt = (int)min((int64_t)kPfThreads, last - c0);
        // per-line strength, profile and shift
        double S = 0.0;
        int pid = -1;
        int64_t shift = 0;
        if (j < cnt) {
            const int64_t i = c0 + j;
            const double nu0 = ln.nu0[i];
            S = pf_strength(ln.s296[i], nu0, ln.elow[i], Tc, qratio);
            const double sig = (nu0 / kLight) * sqrt((kBoltz * Tc) / (ln.mass[i] * kAmu));
            const double gam = (ln.gamma296[i] * pf) * sq;
            pid = pf_nearest(pv.smid, pv.n_sigma, sig) * pv.n_gamma + pf_nearest(pv.gmid, pv.n_gamma, gam);
            shift = (int64_t)rint((nu0 - nu_start) / pv.delta);
            if (!(S >= thr)) S = 0.0;  // item 6: below the threshold
        }
        s_pid[j] = pid;
        s_shift[j] = shift;
        __syncthreads();
        // item 5: runs of equal (profile, shift) keys; a segmented inclusive scan of the
        // strengths leaves each run's sum on its last line
        int head = (j == 0 || j >= cnt || s_pid[j - 1] != pid || s_shift[j - 1] != shift) ? 1 : 0;
        const bool tail = j < cnt && (j == cnt - 1 || s_pid[j + 1] != pid || s_shift[j + 1] != shift);
        double v = S;
        for (int o = 1; o < kPfThreads; o <<= 1) {
            s_S[j] = v;
            s_flag[j] = head;
            __syncthreads();
            if (j >= o && !head) {
                v += s_S[j - o];
                head = s_flag[j - o];
            }
            __syncthreads();
        }
        // each run's last line carries the run; the others drop out
        double eff = (tail && v != 0.0) ? v : 0.0;
        int64_t u0 = 0, two_t = -1, base = 0;
        if (eff != 0.0) {
            const int64_t Tp = pv.ext[pid];
            u0 = k0 * O - shift + Tp;
            const int64_t rho = ((u0 % O) + O) % O;
            const int64_t col0 = (u0 - rho) / O;
            base = pv.off[pid] + rho * pv.rows[pid] + col0;
            two_t = 2 * Tp;
        }
        s_S[j] = eff;
        s_u0[j] = u0;
        s_2t[j] = two_t;
        s_base[j] = base;
        __syncthreads();
        if (k < n_nu) {
            const int64_t jo = (int64_t)j * O;
            for (int q = 0; q < cnt; ++q) {
                const double Sq = s_S[q];
                if (Sq == 0.0) continue;
                const int64_t u = s_u0[q] + jo;
                if (u >= 0 && u <= s_2t[q]) acc += Sq * (double)pv.data[s_base[q] + j];
            }
        }
        __syncthreads();
    }
    if (k < n_nu) out[(size_t)cell * n_nu + k] = (T)acc;
}

}  // namespace bm

using namespace bm;

extern "C" size_t bm_voigt_table_bytes(const bm_voigt_grid* grid) {
    ProfileLayout L;
    return profile_layout(grid, L) == BM_OK ? L.total_bytes : 0;
}

extern "C" int bm_voigt_table_build(const bm_voigt_grid* grid, void* table, size_t table_bytes, void* stream) {
    ProfileLayout L;
    int st = profile_layout(grid, L);
    if (st != BM_OK) return st;
    if (!table) return BM_EINVAL;
    if (table_bytes < L.total_bytes) return BM_ESHAPE;
    const std::vector<char> hdr = layout_header(L);
    hipStream_t s = (hipStream_t)stream;
    BM_CHECK_HIP(hipMemcpyAsync(table, hdr.data(), hdr.size(), hipMemcpyHostToDevice, s));
    BM_CHECK_HIP(hipStreamSynchronize(s));  // the host header buffer ends with this call
    const int64_t total = L.off[L.n];
    if (total > 0) {
        const int64_t blocks = std::min<int64_t>((total + 255) / 256, 1 << 20);
        hipLaunchKernelGGL(k_profile_fill, dim3((unsigned)blocks), dim3(256), 0, s, layout_view(L, table), total,
                           weideman(), (float*)((char*)table + L.data_off));
        BM_CHECK_HIP(hipGetLastError());
    }
    return BM_OK;
}

extern "C" size_t bm_opacity_profiles_workspace(int n_temp) {
    if (n_temp < 1 || n_temp > BM_MAX_TEMPS) return 0;
    return sizeof(double) * pf_workspace_doubles(n_temp);
}

extern "C" int bm_opacity_table_build_profiles(const double* nu0, const double* s296, const double* gamma296,
                                               const double* elow, const double* mass_amu, int64_t n_lines,
                                               const double* temp, int n_temp, const double* p_bar, int n_p,
                                               double nu_start, int n_nu, const bm_voigt_grid* grid,
                                               const void* table, double strength_cutoff, int dtype, void* sigma_out,
                                               void* workspace, size_t workspace_bytes, void* stream) {
    ProfileLayout L;
    int st = profile_layout(grid, L);
    if (st != BM_OK) return st;
    if (!temp || !p_bar || !sigma_out || !table || !workspace) return BM_EINVAL;
    if (n_lines > 0 && (!nu0 || !s296 || !gamma296 || !elow || !mass_amu)) return BM_EINVAL;
    if (n_lines < 0 || n_temp < 1 || n_temp > BM_MAX_TEMPS || n_p < 1 || n_p > BM_MAX_LAYERS || n_nu < 1)
        return BM_ESHAPE;
    if (!std::isfinite(nu_start) || !(strength_cutoff >= 0.0) || !std::isfinite(strength_cutoff)) return BM_EINVAL;
    if (dtype != BM_F32 && dtype != BM_F64) return BM_EINVAL;
    if (workspace_bytes < sizeof(double) * pf_workspace_doubles(n_temp)) return BM_ESHAPE;
    PfCells cg{};
    for (int i = 0; i < n_temp; ++i) {
        if (!(temp[i] > 0.0)) return BM_EINVAL;
        cg.temp[i] = temp[i];
    }
    for (int i = 0; i < n_p; ++i) {
        if (!(p_bar[i] > 0.0)) return BM_EINVAL;
        cg.p_bar[i] = p_bar[i];
    }
    cg.n_t = n_temp;
    cg.n_p = n_p;
    hipStream_t s = (hipStream_t)stream;
    PfLines ln{nu0, s296, gamma296, elow, mass_amu, n_lines};
    double* ws = (double*)workspace;
    hipLaunchKernelGGL(k_line_stats, dim3(kPfStatBlocks, n_temp), dim3(kPfThreads), 0, s, ln, cg, ws);
    BM_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_line_stats_final, dim3(1), dim3(128), 0, s, n_temp, ws);
    BM_CHECK_HIP(hipGetLastError());
    const ProfileView pv = layout_view(L, table);
    dim3 g2((n_nu + kPfThreads - 1) / kPfThreads, n_temp * n_p);
    if (dtype == BM_F32)
        hipLaunchKernelGGL(k_opacity_profiles<float>, g2, dim3(kPfThreads), 0, s, ln, cg, nu_start, L.dnu, n_nu, pv,
                           strength_cutoff, (const double*)ws, (float*)sigma_out);
    else
        hipLaunchKernelGGL(k_opacity_profiles<double>, g2, dim3(kPfThreads), 0, s, ln, cg, nu_start, L.dnu, n_nu,
                           pv, strength_cutoff, (const double*)ws, (double*)sigma_out);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}
