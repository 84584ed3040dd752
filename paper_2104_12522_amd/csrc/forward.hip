// Steps a3-a6 of the forward model on the GPU and the C-ABI entry points that expose
// them: temperature interpolation of the opacity tables and extinction (Sec. 3,
// Sec. 6.1.1), chord optical depth through spherical layers and the transit-depth
// integral over impact parameter (Sec. 6.1), channel binning and chi^2 (Sec. 3).
//
// Hot kernel: k_forward. One workgroup owns 64 consecutive wavenumbers (one per lane)
// of one sample and all of its layers:
//   phase 1  the waves stride over layers; each lane streams the two bracketing
//            temperature rows of every species table (coalesced along wavenumber,
//            non-temporal) plus the CIA rows, and leaves e[l][lane] in LDS;
//   phase 2  8-row blocks of the triangular chord-weight matrix are dealt to waves;
//            a lane keeps 8 optical depths in registers, reads e once per layer from
//            LDS, and the chord weights of a block column arrive as uniform (scalar)
//            loads; each finished optical depth is turned into 1 - exp(-tau) and
//            accumulated in double with its impact-parameter weight;
//   phase 3  the per-wave partial sums are combined in a fixed order;
//   phase 4  the last workgroup of a sample (atomic tile counter) bins the spectrum
//            and forms chi^2 in a fixed order.
#include "bm_forward.h"

#include <vector>

namespace bm {

template <typename T, bool kNonTemporal>
__device__ __forceinline__ T ld_table(const T* p) {
    if constexpr (kNonTemporal)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <typename T, int kWaves, int kS, bool kNonTemporal>
__global__ void __launch_bounds__(kWaves * kWave)
    k_forward(LaunchPlan plan, char* __restrict__ ws, double* __restrict__ depth,
              double* __restrict__ binned, double* __restrict__ chi2) {
    extern __shared__ __align__(16) char smem[];
    const int si = plan.segment_of_tile(blockIdx.x);
    const Segment& sg = plan.seg[si];
    const ModelDev& m = plan.model[sg.model];
    const int local = blockIdx.x - sg.tile_begin;
    const int s_in = local / sg.tiles;
    const int tile = local - s_in * sg.tiles;
    const int b = sg.first + s_in;
    const int L = m.L, Nnu = m.Nnu;
    const RecordView<T> rec(ws + sg.ws_off + (size_t)s_in * sg.rec_bytes, kS, L);

    const int lane = threadIdx.x & (kWave - 1);
    // the wave index is uniform across a wave; readfirstlane lets the compiler keep the
    // layer loops and every per-layer record load on the scalar unit
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int nu = tile * kTileNu + lane;
    const bool valid = nu < Nnu;
    const int nu_c = valid ? nu : Nnu - 1;

    T* es = reinterpret_cast<T*>(smem);                                       // [L][64]
    double* red = reinterpret_cast<double*>(smem + align_up(sizeof(T) * L * kTileNu, 16));
    double* dout = depth + sg.depth_off + (size_t)s_in * Nnu;
    const int flags = rec.hdr->flags;

    if (flags & BM_FLAG_RADIUS) {
        if (wave == 0 && valid) dout[nu] = __builtin_nan("");
    } else {
        // ---- phase 1: extinction into LDS ------------------------------------------
        const T* __restrict__ sig = static_cast<const T*>(m.sigma);
        const T* __restrict__ cia = static_cast<const T*>(m.cia);
        const size_t t_stride = (size_t)L * Nnu;
        const size_t s_stride = (size_t)m.NT * t_stride;
        const bool has_cia = m.NTc > 0;
#pragma unroll 2
        for (int l = wave; l < L; l += kWaves) {
            const T* p = sig + (size_t)rec.kidx[l] * t_stride + (size_t)l * Nnu + nu_c;
            T s0[kS], s1[kS];
#pragma unroll
            for (int i = 0; i < kS; ++i) {
                s0[i] = ld_table<T, kNonTemporal>(p + i * s_stride);
                s1[i] = ld_table<T, kNonTemporal>(p + i * s_stride + t_stride);
            }
            T c0 = T(0), c1 = T(0);
            if (has_cia) {
                const T* c = cia + (size_t)rec.kcidx[l] * Nnu + nu_c;
                c0 = c[0];
                c1 = c[Nnu];
            }
            const T w = rec.w[l];
            T e = T(0);
#pragma unroll
            for (int i = 0; i < kS; ++i) e = fma(rec.afac[i * L + l], fma(w, s1[i] - s0[i], s0[i]), e);
            if (has_cia) e = fma(rec.bfac[l], fma(rec.wc[l], c1 - c0, c0), e);
            es[l * kTileNu + lane] = e;
        }
        __syncthreads();

        // ---- phase 2: chord optical depth, 1 - exp(-tau), impact-parameter sum -------
        double acc = 0.0;
        const int nbu = (L - 1 + kRows - 1) / kRows;  // blocks holding a row j <= L-2
        for (int blk = 0; blk < nbu; ++blk) {
            const int round = blk / kWaves, pos = blk - round * kWaves;
            const int owner = (round & 1) ? (kWaves - 1 - pos) : pos;  // snake: balances work
            if (owner != wave) continue;
            const int j0 = blk * kRows;
            T t[kRows];
#pragma unroll
            for (int r = 0; r < kRows; ++r) t[r] = T(0);
            const T* __restrict__ wcol = rec.wb + (size_t)blk * L * kRows;
            int l = j0;
            // four layers per step: 4 LDS reads and 32 chord weights in flight per wait
            for (; l + 4 <= L; l += 4) {
                T e[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) e[u] = es[(l + u) * kTileNu + lane];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int r = 0; r < kRows; ++r) t[r] = fma(wcol[(l + u) * kRows + r], e[u], t[r]);
            }
            for (; l < L; ++l) {
                const T e = es[l * kTileNu + lane];
#pragma unroll
                for (int r = 0; r < kRows; ++r) t[r] = fma(wcol[l * kRows + r], e, t[r]);
            }
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                const int j = j0 + r;
                if (j <= L - 2) acc += rec.cw[j] * (double)(-dev_expm1(-t[r]));
            }
        }
        red[wave * kTileNu + lane] = acc;
        __syncthreads();
        if (wave == 0) {
            double s = rec.hdr->base;
            for (int w2 = 0; w2 < kWaves; ++w2) s += red[w2 * kTileNu + lane];
            if (valid) dout[nu] = s / rec.hdr->rs2;
        }
    }

    // ---- phase 4: the last tile of this sample bins the spectrum and forms chi^2 ------
    if (binned == nullptr || m.bin_width <= 0) return;
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        int prev = __hip_atomic_fetch_add(&rec.hdr->counter, 1, __ATOMIC_ACQ_REL,
                                          __HIP_MEMORY_SCOPE_AGENT);
        is_last = (prev == sg.tiles - 1);
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    const int bw = m.bin_width;
    const int nbins = Nnu / bw;
    double* bout = binned + sg.bin_off + (size_t)s_in * nbins;
    const bool want_chi2 = (chi2 != nullptr) && m.data && m.err;
    double c2 = 0.0;
    for (int c = threadIdx.x; c < nbins; c += blockDim.x) {
        double s = 0.0;
        for (int q = 0; q < bw; ++q)
            s += __hip_atomic_load(dout + (size_t)c * bw + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double mean = s / bw;
        bout[c] = mean;
        if (want_chi2) {
            const double d = (mean - m.data[c]) / m.err[c];
            c2 += d * d;
        }
    }
    if (want_chi2) {
        // fixed-order reduction: per-thread partials, then thread 0 in index order
        double* part = reinterpret_cast<double*>(smem);
        __syncthreads();
        part[threadIdx.x] = c2;
        __syncthreads();
        if (threadIdx.x == 0) {
            double tot = 0.0;
            for (int i = 0; i < (int)blockDim.x; ++i) tot += part[i];
            chi2[b] = tot;
        }
    }
    if (threadIdx.x == 0) rec.hdr->counter = 0;
}

// ---------------------------------------------------------------------------------------
// standalone step kernels (a3, a4, a5, a6)
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ void k_extinction(ModelDev m, const double* __restrict__ temp, const double* __restrict__ nsp,
                             const double* __restrict__ nh2, T* __restrict__ ext, int32_t* flags) {
    const int l = blockIdx.y;
    const int nu = blockIdx.x * blockDim.x + threadIdx.x;
    const int L = m.L, Nnu = m.Nnu;
    int k, kc = 0;
    double w, wc = 0.0;
    bool clamped = interp_bracket(m.temp, m.NT, temp[l], &k, &w);
    if (m.NTc > 0) clamped |= interp_bracket(m.temp_cia, m.NTc, temp[l], &kc, &wc);
    if (clamped && nu == 0) atomicOr(flags, BM_FLAG_T_CLAMP);
    if (nu >= Nnu) return;
    const T* sig = static_cast<const T*>(m.sigma);
    const size_t t_stride = (size_t)L * Nnu;
    const size_t s_stride = (size_t)m.NT * t_stride;
    double e = 0.0;
    for (int i = 0; i < m.S; ++i) {
        const T* p = sig + i * s_stride + (size_t)k * t_stride + (size_t)l * Nnu + nu;
        double s0 = (double)p[0], s1 = (double)p[t_stride];
        e += nsp[i * L + l] * ((1.0 - w) * s0 + w * s1);
    }
    if (m.NTc > 0) {
        const T* c = static_cast<const T*>(m.cia) + (size_t)kc * Nnu + nu;
        double c0 = (double)c[0], c1 = (double)c[Nnu];
        e += nh2[l] * nh2[l] * ((1.0 - wc) * c0 + wc * c1);
    }
    ext[(size_t)l * Nnu + nu] = (T)e;
}

// tau[j][nu] = sum_{l=j}^{L-2} (s_{j,l+1} - s_{j,l}) (e_l + e_{l+1}); chord lengths in double
template <typename T>
__global__ void k_optical_depth(const double* __restrict__ radius, const T* __restrict__ ext, int L,
                                int Nnu, T* __restrict__ tau) {
    __shared__ double r[BM_MAX_LAYERS];
    for (int i = threadIdx.x; i < L; i += blockDim.x) r[i] = radius[i];
    __syncthreads();
    const int j = blockIdx.y;
    const int nu = blockIdx.x * blockDim.x + threadIdx.x;
    if (nu >= Nnu) return;
    T acc = T(0);
    double s_prev = 0.0;
    for (int l = j; l < L - 1; ++l) {
        const double s_next = half_chord(r[l + 1], r[j]);
        const T ds = (T)(s_next - s_prev);
        acc += ds * (ext[(size_t)l * Nnu + nu] + ext[(size_t)(l + 1) * Nnu + nu]);
        s_prev = s_next;
    }
    tau[(size_t)j * Nnu + nu] = acc;
}

template <typename T>
__global__ void k_transit_depth(const double* __restrict__ radius, const T* __restrict__ tau, int L,
                                int Nnu, double rs2, double* __restrict__ depth) {
    const int nu = blockIdx.x * blockDim.x + threadIdx.x;
    if (nu >= Nnu) return;
    double acc = radius[0] * radius[0];
    double f_lo = -(double)dev_expm1(-tau[nu]);
    for (int j = 0; j < L - 1; ++j) {
        const double f_hi = -(double)dev_expm1(-tau[(size_t)(j + 1) * Nnu + nu]);
        acc += (radius[j + 1] - radius[j]) * (f_lo * radius[j] + f_hi * radius[j + 1]);
        f_lo = f_hi;
    }
    depth[nu] = acc / rs2;
}

__global__ void k_bin_chi2(const double* __restrict__ depth, int Nnu, int bw, const double* __restrict__ data,
                           const double* __restrict__ err, double* __restrict__ binned,
                           double* __restrict__ chi2) {
    __shared__ double part[256];
    const int b = blockIdx.x;
    const int nbins = Nnu / bw;
    double c2 = 0.0;
    for (int c = threadIdx.x; c < nbins; c += blockDim.x) {
        double s = 0.0;
        for (int q = 0; q < bw; ++q) s += depth[(size_t)b * Nnu + (size_t)c * bw + q];
        const double mean = s / bw;
        if (binned) binned[(size_t)b * nbins + c] = mean;
        if (data && err) {
            const double d = (mean - data[c]) / err[c];
            c2 += d * d;
        }
    }
    part[threadIdx.x] = c2;
    __syncthreads();
    if (threadIdx.x == 0 && chi2 && data && err) {
        double tot = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) tot += part[i];
        chi2[b] = tot;
    }
}

// ---------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------
int validate_model(const bm_model& m, bool need_tables) {
    if (m.dtype != BM_F32 && m.dtype != BM_F64) return BM_EINVAL;
    if (m.n_species < 1 || m.n_species > BM_MAX_SPECIES) return BM_ESHAPE;
    if (m.n_layers < 2 || m.n_layers > BM_MAX_LAYERS) return BM_ESHAPE;
    if (m.tp_mode != BM_TP_ISOTHERMAL && m.tp_mode != BM_TP_LINE2013) return BM_EINVAL;
    if (!m.p_bar) return BM_EINVAL;
    if (!need_tables) return BM_OK;
    if (m.n_nu < 1 || m.n_temp < 2 || m.n_temp > BM_MAX_TEMPS) return BM_ESHAPE;
    if (m.n_temp_cia != 0 && (m.n_temp_cia < 2 || m.n_temp_cia > BM_MAX_TEMPS)) return BM_ESHAPE;
    if (!m.sigma || !m.temp) return BM_EINVAL;
    if (m.n_temp_cia > 0 && (!m.cia || !m.temp_cia)) return BM_EINVAL;
    if (m.bin_width < 0) return BM_ESHAPE;
    if (m.bin_width > 0 && m.n_nu / m.bin_width < 1) return BM_ESHAPE;
    return BM_OK;
}

ModelDev to_device_view(const bm_model& m) {
    ModelDev d{};
    d.sigma = m.sigma;
    d.temp = m.temp;
    d.cia = m.cia;
    d.temp_cia = m.temp_cia;
    d.p_bar = m.p_bar;
    d.data = m.data;
    d.err = m.err;
    d.S = m.n_species;
    d.NT = m.n_temp;
    d.L = m.n_layers;
    d.Nnu = m.n_nu;
    d.NTc = m.n_temp_cia;
    d.tp_mode = m.tp_mode;
    d.bin_width = m.bin_width;
    d.nb = row_blocks(m.n_layers);
    for (int i = 0; i < BM_MAX_SPECIES; ++i) d.mass[i] = m.mass_amu[i];
    d.pl = m.planet;
    return d;
}

static size_t record_bytes(const bm_model& m) {
    return m.dtype == BM_F32 ? RecordLayout<float>(m.n_species, m.n_layers).total
                             : RecordLayout<double>(m.n_species, m.n_layers).total;
}

// Split a batch into launch plans of at most kMaxSegments same-model runs.
struct HostPlan {
    std::vector<LaunchPlan> plans;
    std::vector<int> first_sample;   // first sample of each plan
    std::vector<int> n_samples;      // samples of each plan
    size_t ws_bytes = 0;
    int max_L = 0;
    int n_species = 0;
};

static int build_plans(const bm_model* models, int n_models, const int32_t* instance, int B,
                       HostPlan& hp) {
    if (!models || n_models < 1 || n_models > kMaxModels || B < 0) return BM_EINVAL;
    const int dtype = models[0].dtype;
    for (int i = 0; i < n_models; ++i) {
        int st = validate_model(models[i], true);
        if (st != BM_OK) return st;
        if (models[i].dtype != dtype) return BM_EINVAL;
        // one launch is specialised on the species count
        if (models[i].n_species != models[0].n_species) return BM_ESHAPE;
    }
    hp.n_species = models[0].n_species;
    size_t ws = 0, depth_off = 0, bin_off = 0;
    int b = 0;
    while (b < B) {
        LaunchPlan lp{};
        for (int i = 0; i < n_models; ++i) lp.model[i] = to_device_view(models[i]);
        int first_of_plan = b;
        int tiles = 0;
        while (b < B && lp.n_seg < kMaxSegments) {
            const int mi = instance ? instance[b] : 0;
            if (mi < 0 || mi >= n_models) return BM_EINVAL;
            int e = b + 1;
            while (e < B && (instance ? instance[e] : 0) == mi) ++e;
            const bm_model& md = models[mi];
            Segment& s = lp.seg[lp.n_seg++];
            s.model = mi;
            s.first = b - first_of_plan;
            s.count = e - b;
            s.tiles = (md.n_nu + kTileNu - 1) / kTileNu;
            s.tile_begin = tiles;
            s.ws_off = ws;
            s.rec_bytes = record_bytes(md);
            s.depth_off = depth_off;
            s.bin_off = bin_off;
            tiles += s.count * s.tiles;
            ws += s.rec_bytes * s.count;
            depth_off += (size_t)md.n_nu * s.count;
            bin_off += (size_t)(md.bin_width > 0 ? md.n_nu / md.bin_width : 0) * s.count;
            if (md.n_layers > hp.max_L) hp.max_L = md.n_layers;
            b = e;
        }
        lp.total_tiles = tiles;
        hp.plans.push_back(lp);
        hp.first_sample.push_back(first_of_plan);
        hp.n_samples.push_back(b - first_of_plan);
    }
    hp.ws_bytes = ws;
    return BM_OK;
}

constexpr int kFwdWaves = 8;

template <typename T>
static size_t forward_lds_bytes(int max_L) {
    size_t a = align_up(sizeof(T) * max_L * kTileNu, 16) + sizeof(double) * kFwdWaves * kTileNu;
    size_t b = sizeof(double) * kFwdWaves * kTileNu;  // chi^2 partials reuse the front
    return a > b ? a : b;
}

template <typename T>
static int launch_forward(const HostPlan& hp, const double* params, int stride, double* depth,
                          double* binned, double* chi2, int32_t* flags, char* ws, hipStream_t st) {
    const size_t lds = forward_lds_bytes<T>(hp.max_L);
    if (lds > 64 * 1024) return BM_ESHAPE;
    for (size_t p = 0; p < hp.plans.size(); ++p) {
        const LaunchPlan& lp = hp.plans[p];
        const int b0 = hp.first_sample[p];
        const int nb = hp.n_samples[p];
        // Segment offsets inside a plan are absolute (workspace, depth, binned); sample
        // indices are relative to the plan, so params/flags/chi2 are shifted here.
        hipLaunchKernelGGL((k_atm_prep<T>), dim3(nb), dim3(kAtmThreads), 0, st, lp,
                           params + (size_t)b0 * stride, stride, ws, flags + b0);
        BM_CHECK_HIP(hipGetLastError());
        double* c2 = chi2 ? chi2 + b0 : nullptr;
        const dim3 grid(lp.total_tiles), block(kFwdWaves * kWave);
        switch (hp.n_species) {
#define BM_FWD_CASE(NS)                                                                              \
    case NS:                                                                                        \
        hipLaunchKernelGGL((k_forward<T, kFwdWaves, NS, true>), grid, block, lds, st, lp, ws, depth, \
                           binned, c2);                                                             \
        break;
            BM_FWD_CASE(1) BM_FWD_CASE(2) BM_FWD_CASE(3) BM_FWD_CASE(4)
            BM_FWD_CASE(5) BM_FWD_CASE(6) BM_FWD_CASE(7) BM_FWD_CASE(8)
#undef BM_FWD_CASE
            default: return BM_ESHAPE;
        }
        BM_CHECK_HIP(hipGetLastError());
    }
    return BM_OK;
}

}  // namespace bm

// =========================================================================================
// C ABI
// =========================================================================================
using namespace bm;

extern "C" const char* bm_status_string(int status) {
    switch (status) {
        case BM_OK: return "ok";
        case BM_EINVAL: return "invalid argument";
        case BM_ESHAPE: return "unsupported or inconsistent shape";
        case BM_EHIP: return "HIP runtime error";
        case BM_ENOSPACE: return "workspace too small";
        default: return "unknown status";
    }
}

extern "C" int bm_version(void) { return 100; }

extern "C" int bm_n_params(const bm_model* model) {
    if (!model) return BM_EINVAL;
    return (model->tp_mode == BM_TP_ISOTHERMAL ? 1 : 5) + model->n_species + 1;
}

extern "C" int bm_extinction(const bm_model* model, const double* temp, const double* n_species,
                             const double* n_h2, void* ext, int32_t* flags, void* stream) {
    if (!model || !temp || !n_species || !ext || !flags) return BM_EINVAL;
    int st = validate_model(*model, true);
    if (st != BM_OK) return st;
    if (model->n_temp_cia > 0 && !n_h2) return BM_EINVAL;
    ModelDev m = to_device_view(*model);
    dim3 grid((model->n_nu + 255) / 256, model->n_layers);
    if (model->dtype == BM_F32)
        hipLaunchKernelGGL(k_extinction<float>, grid, dim3(256), 0, (hipStream_t)stream, m, temp, n_species,
                           n_h2, (float*)ext, flags);
    else
        hipLaunchKernelGGL(k_extinction<double>, grid, dim3(256), 0, (hipStream_t)stream, m, temp, n_species,
                           n_h2, (double*)ext, flags);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

extern "C" int bm_optical_depth(const double* radius, const void* ext, int L, int n_nu, int dtype,
                                void* tau, void* stream) {
    if (!radius || !ext || !tau) return BM_EINVAL;
    if (L < 2 || L > BM_MAX_LAYERS || n_nu < 1) return BM_ESHAPE;
    dim3 grid((n_nu + 255) / 256, L);
    if (dtype == BM_F32)
        hipLaunchKernelGGL(k_optical_depth<float>, grid, dim3(256), 0, (hipStream_t)stream, radius,
                           (const float*)ext, L, n_nu, (float*)tau);
    else if (dtype == BM_F64)
        hipLaunchKernelGGL(k_optical_depth<double>, grid, dim3(256), 0, (hipStream_t)stream, radius,
                           (const double*)ext, L, n_nu, (double*)tau);
    else
        return BM_EINVAL;
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

extern "C" int bm_transit_depth(const double* radius, const void* tau, int L, int n_nu, int dtype,
                                double rs_cm, double* depth, void* stream) {
    if (!radius || !tau || !depth) return BM_EINVAL;
    if (L < 2 || L > BM_MAX_LAYERS || n_nu < 1) return BM_ESHAPE;
    if (!(rs_cm > 0.0)) return BM_EINVAL;
    dim3 grid((n_nu + 255) / 256);
    if (dtype == BM_F32)
        hipLaunchKernelGGL(k_transit_depth<float>, grid, dim3(256), 0, (hipStream_t)stream, radius,
                           (const float*)tau, L, n_nu, rs_cm * rs_cm, depth);
    else if (dtype == BM_F64)
        hipLaunchKernelGGL(k_transit_depth<double>, grid, dim3(256), 0, (hipStream_t)stream, radius,
                           (const double*)tau, L, n_nu, rs_cm * rs_cm, depth);
    else
        return BM_EINVAL;
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

extern "C" int bm_bin_chi2(const double* depth, int B, int n_nu, int bin_width, const double* data,
                           const double* err, double* binned, double* chi2, void* stream) {
    if (!depth || (!binned && !chi2)) return BM_EINVAL;
    if (B < 0 || n_nu < 1 || bin_width < 1 || n_nu / bin_width < 1) return BM_ESHAPE;
    if (chi2 && (!data || !err)) return BM_EINVAL;
    if (B == 0) return BM_OK;
    hipLaunchKernelGGL(k_bin_chi2, dim3(B), dim3(256), 0, (hipStream_t)stream, depth, n_nu, bin_width, data,
                       err, binned, chi2);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

extern "C" size_t bm_workspace_size(const bm_model* models, int n_models, const int32_t* instance, int B) {
    HostPlan hp;
    if (build_plans(models, n_models, instance, B, hp) != BM_OK) return 0;
    return hp.ws_bytes;
}

extern "C" int bm_forward_batch(const bm_model* models, int n_models, const int32_t* instance,
                                const double* params, int param_stride, int B, double* depth,
                                double* binned, double* chi2, int32_t* flags, void* workspace,
                                size_t workspace_bytes, void* stream) {
    if (!models || !params || !depth || !flags || !workspace) return BM_EINVAL;
    HostPlan hp;
    int st = build_plans(models, n_models, instance, B, hp);
    if (st != BM_OK) return st;
    if (B == 0) return BM_OK;
    for (int i = 0; i < n_models; ++i) {
        if (param_stride < bm_n_params(&models[i])) return BM_ESHAPE;
        if (binned && models[i].bin_width <= 0) return BM_EINVAL;
        if (chi2 && (!models[i].data || !models[i].err)) return BM_EINVAL;
    }
    if (chi2 && !binned) return BM_EINVAL;
    if (workspace_bytes < hp.ws_bytes) return BM_ENOSPACE;
    const hipStream_t s = (hipStream_t)stream;
    if (models[0].dtype == BM_F32)
        return launch_forward<float>(hp, params, param_stride, depth, binned, chi2, flags, (char*)workspace, s);
    return launch_forward<double>(hp, params, param_stride, depth, binned, chi2, flags, (char*)workspace, s);
}
