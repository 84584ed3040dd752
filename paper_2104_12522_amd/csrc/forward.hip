// Host side of the forward model and the C-ABI entry points (steps a3-a6): the launch
// plans of the fused kernel (fwd_kernel.h), the per-sample chi^2 reduction, the
// standalone step kernels, the autotuner and the kernel-timing hook.
#include "fwd_kernel.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace bm {

// the fused kernel's launchers are instantiated in fwd_f32_nt.hip, fwd_f32_t.hip,
// fwd_f32_pipe_nt.hip, fwd_f32_pipe_t.hip and fwd_f64.hip (compiled in parallel)
#define BM_FWD_EXTERN(T, W, NT, MODE)                                                                  \
    extern template int launch_k_forward<T, W, NT, MODE>(const HostPlan&, const LaunchPlan&, size_t, char*, \
                                                          const int32_t*, double*, double*, double*,      \
                                                          const int32_t*, const int32_t*, int,            \
                                                          hipStream_t, hipEvent_t, hipEvent_t);
BM_FWD_EXTERN(float, 8, true, 1)
BM_FWD_EXTERN(float, 8, true, 0)
BM_FWD_EXTERN(float, 8, false, 1)
BM_FWD_EXTERN(float, 8, false, 0)
BM_FWD_EXTERN(float, 8, true, 2)
BM_FWD_EXTERN(float, 8, false, 2)
BM_FWD_EXTERN(double, 8, true, 0)
#undef BM_FWD_EXTERN
// chi^2 of each sample: the tiles' partials summed in a fixed tree (one workgroup per
// sample, after the forward kernel: the kernel boundary orders the partial writes)
template <typename T>
__global__ void __launch_bounds__(256)
    k_chi2_reduce(LaunchPlan plan, char* __restrict__ ws, const int32_t* __restrict__ active, double* __restrict__ chi2) {
    __shared__ double cp[256];
    const int b = blockIdx.x;
    if (active && !active[b]) return;
    const Segment& sg = plan.seg[plan.segment_of_sample(b)];
    const ModelDev& m = plan.model[sg.model];
    const RecordView<T> rec(ws + sg.ws_off + (size_t)(b - sg.first) * sg.rec_bytes, m.S, m.L);
    double v = 0.0;
    for (int i = threadIdx.x; i < sg.tiles; i += 256) v += rec.chi2part[i];
    cp[threadIdx.x] = v;
    __syncthreads();
    for (int half = 128; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) cp[threadIdx.x] += cp[threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x == 0) chi2[b] = cp[0];
}

// The same sum for a single-segment plan, from plain pointers: sample b's n partials
// start at part + b * stride (doubles). Each wave sums its lanes' partials with shuffles
// (a fixed tree, so the result does not depend on timing), then one thread adds the
// waves' sums in order.
__global__ void __launch_bounds__(256)
    k_chi2_sum(const double* __restrict__ part, size_t stride, int n, const int32_t* __restrict__ active,
               double* __restrict__ chi2) {
    __shared__ double ws[4];
    const int b = blockIdx.x;
    const double* p = part + (size_t)b * stride;
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) v += p[i];
    if (active && !active[b]) return;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) ws[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) chi2[b] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
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
        const double* c = static_cast<const double*>(m.cia) + (size_t)kc * Nnu + nu;
        double c0 = c[0], c1 = c[Nnu];
        e += nh2[l] * nh2[l] * ((1.0 - wc) * c0 + wc * c1);
    }
    if (m.rayleigh) e += nh2[l] * rayleigh_h2_xsec(m.nu_start + m.dnu * nu);
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
    double f_lo = (double)dev_absorbed(tau[nu]);
    for (int j = 0; j < L - 1; ++j) {
        const double f_hi = (double)dev_absorbed(tau[(size_t)(j + 1) * Nnu + nu]);
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
    if (m.rayleigh && !(m.dnu > 0.0 && m.nu_start + m.dnu * (m.n_nu - 1) > 0.0 && m.nu_start > 0.0))
        return BM_EINVAL;
    if (m.geometry != BM_GEOM_TRANSIT && m.geometry != BM_GEOM_ECLIPSE) return BM_EINVAL;
    if (m.geometry == BM_GEOM_ECLIPSE && (m.cloud || m.tau_max > 0.0 || !(m.dnu > 0.0) || !(m.nu_start > 0.0)))
        return BM_EINVAL;
    if (m.sigma_tiles && (m.tile_w < 1 || m.tile_w > kTileNu)) return BM_EINVAL;
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
    d.tau_max = (m.tau_max > 0.0) ? m.tau_max : __builtin_huge_val();
    d.nu_start = m.nu_start;
    d.dnu = m.dnu;
    d.rayleigh = m.rayleigh ? 1 : 0;
    d.cloud = m.cloud ? 1 : 0;
    d.geometry = m.geometry;
    d.sigma_tiles = m.sigma_tiles;
    d.tile_w = m.sigma_tiles ? m.tile_w : 0;
    return d;
}

// ---- tile-major copy of the opacity tables ---------------------------------------------
// out[s][k][t][l][c] = sigma[s][k][l][min(t tw + c, Nnu - 1)], c < tw: one element per
// thread, consecutive threads write consecutive elements.
template <typename T>
__global__ void __launch_bounds__(256)
    k_sigma_tiles(const T* __restrict__ sigma, int L, int Nnu, int tw, int n_tiles, size_t n_rows,
                  T* __restrict__ out) {
    const size_t total = n_rows * (size_t)n_tiles * L * tw;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (size_t)gridDim.x * 256) {
        const int c = (int)(i % tw);
        size_t q = i / tw;
        const int l = (int)(q % L);
        q /= L;
        const int t = (int)(q % n_tiles);
        const size_t sk = q / n_tiles;  // species-major (species, temperature) row index
        const int nu = min(t * tw + c, Nnu - 1);
        out[i] = sigma[(sk * L + l) * (size_t)Nnu + nu];
    }
}

static size_t sigma_tiles_bytes(const bm_model& m, int tile_w) {
    const size_t n_tiles = (size_t)(m.n_nu + tile_w - 1) / tile_w;
    return (size_t)m.n_species * m.n_temp * n_tiles * m.n_layers * tile_w *
           (m.dtype == BM_F32 ? sizeof(float) : sizeof(double));
}

static size_t record_bytes(const bm_model& m, int tiles) {
    return m.dtype == BM_F32 ? record_bytes_t<float>(m.n_species, m.n_layers, tiles)
                             : record_bytes_t<double>(m.n_species, m.n_layers, tiles);
}


// slices of the record preparation per sample: enough workgroups to spread the chord
// weights of a single spectrum over the chip, fewer when the batch fills it anyway
static int prep_slices(const HostPlan& hp, int nb) {
    int want = (int)((hp.max_entries + 255) / 256);
    int cap = nb > 0 ? 2048 / nb : 1;
    if (cap < 1) cap = 1;
    if (want > cap) want = cap;
    if (want > 64) want = 64;
    return want < 1 ? 1 : want;
}

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
        // one launch is specialised on the presence of CIA
        if ((models[i].n_temp_cia > 0) != (models[0].n_temp_cia > 0)) return BM_ESHAPE;
        if (models[i].geometry != models[0].geometry) return BM_EINVAL;
    }
    hp.geometry = models[0].geometry;
    hp.n_species = models[0].n_species;
    hp.cia = models[0].n_temp_cia > 0;
    size_t ws = 0, depth_off = 0, bin_off = 0;
    int b = 0;
    while (b < B) {
        LaunchPlan lp{};
        lp.prio_from = INT_MAX;  // set per launch
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
            s.fused_bins = (md.geometry == BM_GEOM_TRANSIT && md.bin_width > 0 && md.bin_width <= kTileNu) ? 1 : 0;
            s.tile_w = s.fused_bins ? (kTileNu / md.bin_width) * md.bin_width : kTileNu;
            s.tiles = (md.n_nu + s.tile_w - 1) / s.tile_w;
            s.tiles_per_xcd = (s.tiles + kXcds - 1) / kXcds;
            s.tile_begin = tiles;
            s.ws_off = ws;
            s.rec_bytes = record_bytes(md, s.tiles);
            s.depth_off = depth_off;
            s.bin_off = bin_off;
            tiles += segment_wgs(s.count, s.tiles);
            ws += s.rec_bytes * s.count;
            depth_off += (size_t)md.n_nu * s.count;
            bin_off += (size_t)(md.bin_width > 0 ? md.n_nu / md.bin_width : 0) * s.count;
            if (md.n_layers > hp.max_L) hp.max_L = md.n_layers;
            if (md.n_temp_cia > hp.max_ntc) hp.max_ntc = md.n_temp_cia;
            const size_t ent = md.dtype == BM_F32 ? chord_weight_entries<float>(md.n_layers)
                                                  : chord_weight_entries<double>(md.n_layers);
            if (ent > hp.max_entries) hp.max_entries = ent;
            b = e;
        }
        lp.total_wgs = tiles;
        lp.max_ntc = 0;
        for (int i = 0; i < n_models; ++i)
            if (models[i].n_temp_cia > lp.max_ntc) lp.max_ntc = models[i].n_temp_cia;
        if (lp.max_ntc > hp.max_ntc) hp.max_ntc = lp.max_ntc;
        hp.plans.push_back(lp);
        hp.first_sample.push_back(first_of_plan);
        hp.n_samples.push_back(b - first_of_plan);
    }
    // the list of requested samples of a masked call (k_active_list), then its count
    hp.list_off = align_up(ws, 256);
    hp.ws_bytes = hp.list_off + sizeof(int32_t) * ((size_t)B + 1);
    hp.total_samples = B;
    return BM_OK;
}

// Masked calls of one run of samples: the requested samples' indices in ascending order,
// list[0 .. n), and n = list[B], written by one workgroup (a ballot scan per block of
// 1024 samples), so that the forward kernel's grid can cover a few sample slots per tile
// instead of every sample. Graph-safe: it writes every entry it later reads.
constexpr int kCompactSlots = 16;
constexpr int kCompactSlotsPipe = 4;  // pipelined launches: two workgroups per CU
__global__ void __launch_bounds__(1024)
    k_active_list(const int32_t* __restrict__ active, int B, int32_t* __restrict__ list) {
    __shared__ int wsum[1024 / kWave];
    __shared__ int base;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    for (int b0 = 0; b0 < B; b0 += 1024) {
        const int b = b0 + threadIdx.x;
        const bool on = b < B && active[b] != 0;
        const unsigned long long bal = __ballot(on);
        if (lane == 0) wsum[w] = __popcll(bal);
        __syncthreads();
        int off = base;
        for (int q = 0; q < w; ++q) off += wsum[q];
        if (on) list[off + __popcll(bal & ((1ull << lane) - 1))] = b;
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (int q = 0; q < 1024 / kWave; ++q) t += wsum[q];
            base += t;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) list[B] = base;
}

// Launch configurations of the fused forward kernel that the autotuner chooses from:
// table rows loaded non-temporally (streamed once: one spectrum) or through the caches
// (rows shared by the samples of a tile in a batch); the FP32 chord weights copied into
// LDS at kernel start (short phase 2, more LDS per workgroup), optionally with phases 1
// and 2 interleaved by 16-layer stages, or streamed from L2 in phase 2 (more workgroups
// per CU).
struct FwdConfig {
    int waves;
    bool nontemporal;
    int mode;  // kModeStreamed, kModeStaged, kModePipelined
    const char* name;
};
constexpr FwdConfig kFwdConfigs[] = {
    {8, true, kModeStaged, "non-temporal table loads, chord weights staged in LDS"},
    {8, false, kModeStaged, "cached table loads, chord weights staged in LDS"},
    {8, true, kModeStreamed, "non-temporal table loads, chord weights streamed from L2"},
    {8, false, kModeStreamed, "cached table loads, chord weights streamed from L2"},
    {8, true, kModePipelined, "non-temporal table loads, staged chord weights, pipelined stages"},
    {8, false, kModePipelined, "cached table loads, staged chord weights, pipelined stages"},
};
constexpr int kNumFwdConfigs = sizeof(kFwdConfigs) / sizeof(kFwdConfigs[0]);

// the configuration with the same table loads in another phase-2 mode
static int config_with_mode(int cfg, int mode) {
    for (int c = 0; c < kNumFwdConfigs; ++c)
        if (kFwdConfigs[c].nontemporal == kFwdConfigs[cfg].nontemporal && kFwdConfigs[c].mode == mode) return c;
    return cfg;
}
// the configuration with the same phase-2 mode and cached table loads
static int config_cached(int cfg) {
    for (int c = 0; c < kNumFwdConfigs; ++c)
        if (!kFwdConfigs[c].nontemporal && kFwdConfigs[c].mode == kFwdConfigs[cfg].mode) return c;
    return cfg;
}

// dynamic LDS of a launch; the staged modes add their static staging arrays
template <typename T>
static size_t forward_lds_bytes(int max_L, int waves, int max_ntc, int mode) {
    return FwdLds<T>(max_L, waves, max_ntc, mode == kModePipelined).total;
}
static size_t static_lds_bytes(int mode) {
    if (mode == kModeStaged) return sizeof(float) * (kStageMaxFloats + 4 * kWave);
    if (mode == kModePipelined) return sizeof(float) * (kPipeMaxFloats + 4 * kWave);
    return 0;
}

// Dynamic LDS above 64 KB must be enabled per kernel; the device limit is queried once.
static size_t device_lds_limit() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64 * 1024;
    if (!cached[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 64 * 1024;
        cached[dev] = v;
    }
    return (size_t)cached[dev];
}

// Compute units of the current device, queried once per device (0 if the query fails: the
// fused kernel then skips its dispatch-round heuristics).
int device_cu_count() {
    static std::atomic<int> cached[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    int v = cached[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = -1;
        cached[dev].store(v, std::memory_order_relaxed);
    }
    return v > 0 ? v : 0;
}

// Raise a kernel's dynamic-LDS ceiling once per device (hipFuncSetAttribute is host work
// that the per-call path should not repeat).
int ensure_dynamic_lds(const void* fn, size_t bytes) {
    if (bytes <= 48 * 1024) return BM_OK;
    struct Entry { const void* fn; int dev; size_t bytes; };
    static Entry cache[256];
    static int n_cache = 0;
    static std::mutex mu;
    int dev = 0;
    BM_CHECK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < n_cache; ++i)
        if (cache[i].fn == fn && cache[i].dev == dev && cache[i].bytes >= bytes) return BM_OK;
    BM_CHECK_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    if (n_cache < 256) cache[n_cache++] = Entry{fn, dev, bytes};
    return BM_OK;
}

// ---- kernel timing (measurement hook) -------------------------------------------------
// While a session is open, every launch of the fused kernel outside graph capture carries
// a pair of timing events that its dispatch records at the kernel's start and end.
struct TimingSession {
    std::vector<hipEvent_t> ev;
    int cap = 0, used = 0;
};
static std::mutex g_timing_mu;
static TimingSession* g_timing = nullptr;

static void timing_slot(hipStream_t st, hipEvent_t* e0, hipEvent_t* e1) {
    *e0 = *e1 = nullptr;
    std::lock_guard<std::mutex> lock(g_timing_mu);
    if (!g_timing || g_timing->used >= g_timing->cap) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    const int i = g_timing->used++;
    *e0 = g_timing->ev[2 * i];
    *e1 = g_timing->ev[2 * i + 1];
}

template <typename T>
static int launch_forward(const HostPlan& hp, int cfg, const double* params, int stride, const int32_t* active,
                          double* depth, double* binned, double* chi2, int32_t* flags, char* ws, hipStream_t st) {
    // FP64 (the parity mode) has the default configuration only
    if (cfg < 0 || cfg >= kNumFwdConfigs) cfg = 0;
    if (sizeof(T) == 8) cfg = config_with_mode(0, kModeStreamed);
    // modes that do not fit the batch's layers fall back: pipelined -> staged -> streamed
    auto fits = [&](int c) {
        const int md = kFwdConfigs[c].mode;
        if (md == kModePipelined && hp.max_L > kPipeMaxLayers) return false;
        if (md == kModeStaged && hp.max_L > kStageMaxLayers) return false;
        return forward_lds_bytes<T>(hp.max_L, kFwdConfigs[c].waves, hp.max_ntc, md) + static_lds_bytes(md) <=
               device_lds_limit();
    };
    if (!fits(cfg) && kFwdConfigs[cfg].mode == kModePipelined) cfg = config_with_mode(cfg, kModeStaged);
    if (!fits(cfg)) cfg = config_with_mode(cfg, kModeStreamed);
    if (!fits(cfg)) return BM_ESHAPE;
    // a masked FP32 transit call of one run of samples launches the forward kernel over the
    // list of requested samples (kCompactSlots slots per tile) instead of every sample, with
    // cached table loads (the compacted kernels exist for those) and, where they fit, chord
    // weights staged in LDS: in the compacted kernel they beat weights streamed from L2 at
    // every requested count measured (1-200 of 256 samples, config-2 shapes: 9-20 % less)
    const int B = hp.total_samples;
    const bool compact = sizeof(T) == 4 && active && hp.geometry == BM_GEOM_TRANSIT && hp.plans.size() == 1 &&
                         hp.plans[0].n_seg == 1 && B > kCompactSlots;
    if (compact) {
        cfg = config_cached(cfg);
        if (kFwdConfigs[cfg].mode == kModeStreamed && fits(config_with_mode(cfg, kModeStaged)))
            cfg = config_with_mode(cfg, kModeStaged);
    }
    const size_t lds = forward_lds_bytes<T>(hp.max_L, kFwdConfigs[cfg].waves, hp.max_ntc, kFwdConfigs[cfg].mode);
    int32_t* list = compact ? reinterpret_cast<int32_t*>(ws + hp.list_off) : nullptr;
    // the record preparation builds the list itself for up to kPrepListMax samples (one
    // launch fewer); larger batches take the list kernel first
    const bool prep_builds = compact && B <= kPrepListMax && kAtmThreads * (kPrepListMax / kAtmThreads) == kPrepListMax;
    if (compact && !prep_builds) {
        hipLaunchKernelGGL(k_active_list, dim3(1), dim3(1024), 0, st, active, B, list);
        BM_CHECK_HIP(hipGetLastError());
    }
    const int32_t* list_n = compact ? list + B : nullptr;
    const int slots = compact ? (kFwdConfigs[cfg].mode == kModePipelined ? kCompactSlotsPipe : kCompactSlots) : 0;
    for (size_t p = 0; p < hp.plans.size(); ++p) {
        const LaunchPlan& lp = hp.plans[p];
        const int b0 = hp.first_sample[p];
        const int nb = hp.n_samples[p];
        // Segment offsets inside a plan are absolute (workspace, depth, binned); sample
        // indices are relative to the plan, so params/flags/chi2 are shifted here.
        const int32_t* act = active ? active + b0 : nullptr;
        {
            // one run of samples: its model moves to slot 0 (fixed argument offsets)
            LaunchPlan lp1 = lp;
            const bool single = lp.n_seg == 1;
            if (single) {
                lp1.model[0] = lp.model[lp.seg[0].model];
                lp1.seg[0].model = 0;
            }
            // a compacted call prepares the records of its requested samples only, in a few
            // sample slots that take the list's entries in turn
            const int n_prep = compact ? kCompactSlots : nb;
            const dim3 grid(n_prep, prep_slices(hp, n_prep));
            const double* pp = params + (size_t)b0 * stride;
            if (single && act)
                hipLaunchKernelGGL((k_atm_prep<T, true, true>), grid, dim3(kAtmThreads), 0, st, lp1, pp, stride, act, ws,
                                   flags + b0, list, list_n, prep_builds ? B : 0);
            else if (single)
                hipLaunchKernelGGL((k_atm_prep<T, true, false>), grid, dim3(kAtmThreads), 0, st, lp1, pp, stride, act, ws,
                                   flags + b0, nullptr, nullptr, 0);
            else if (act)
                hipLaunchKernelGGL((k_atm_prep<T, false, true>), grid, dim3(kAtmThreads), 0, st, lp1, pp, stride, act, ws,
                                   flags + b0, list, list_n, prep_builds ? B : 0);
            else
                hipLaunchKernelGGL((k_atm_prep<T, false, false>), grid, dim3(kAtmThreads), 0, st, lp1, pp, stride, act, ws,
                                   flags + b0, nullptr, nullptr, 0);
        }
        BM_CHECK_HIP(hipGetLastError());
        double* c2 = chi2 ? chi2 + b0 : nullptr;
        int code;
        if (hp.geometry == BM_GEOM_ECLIPSE) {
            for (int si = 0; si < lp.n_seg; ++si) {
                code = launch_k_emission<T>(lp, si, ws, act, depth, st);
                if (code != BM_OK) return code;
            }
        } else {
        hipEvent_t e0, e1;
        timing_slot(st, &e0, &e1);
        if constexpr (sizeof(T) == 8) {
            code = launch_k_forward<T, 8, true, kModeStreamed>(hp, lp, lds, ws, act, depth, binned, c2, list, list_n,
                                                              slots, st, e0, e1);
        } else {
#define BM_CFG(NT, MODE) \
    launch_k_forward<T, 8, NT, MODE>(hp, lp, lds, ws, act, depth, binned, c2, list, list_n, slots, st, e0, e1)
            switch (cfg) {
                case 1: code = BM_CFG(false, kModeStaged); break;
                case 2: code = BM_CFG(true, kModeStreamed); break;
                case 3: code = BM_CFG(false, kModeStreamed); break;
                case 4: code = BM_CFG(true, kModePipelined); break;
                case 5: code = BM_CFG(false, kModePipelined); break;
                default: code = BM_CFG(true, kModeStaged); break;
            }
#undef BM_CFG
        }
        if (code != BM_OK) return code;
        }
        if (c2 && binned) {
            bool any_fused = false;
            for (int si = 0; si < lp.n_seg; ++si) any_fused |= lp.seg[si].fused_bins != 0;
            if (any_fused && lp.n_seg == 1) {
                // records are rec_bytes apart; the partials sit at a fixed offset in each
                const Segment& sg = lp.seg[0];
                const ModelDev& m = lp.model[sg.model];
                const char* base = ws + sg.ws_off;
                const double* part0 = RecordView<T>(const_cast<char*>(base), m.S, m.L).chi2part;
                hipLaunchKernelGGL(k_chi2_sum, dim3(nb), dim3(256), 0, st, part0, sg.rec_bytes / sizeof(double),
                                   sg.tiles, act, c2);
                BM_CHECK_HIP(hipGetLastError());
            } else if (any_fused) {
                hipLaunchKernelGGL((k_chi2_reduce<T>), dim3(nb), dim3(256), 0, st, lp, ws, act, c2);
                BM_CHECK_HIP(hipGetLastError());
            }
        }
        // channels wider than a tile: a separate binning pass per run of samples
        if (binned) {
            for (int si = 0; si < lp.n_seg; ++si) {
                const Segment& sg = lp.seg[si];
                if (sg.fused_bins) continue;
                const ModelDev& m = lp.model[sg.model];
                hipLaunchKernelGGL(k_bin_chi2, dim3(sg.count), dim3(256), 0, st, depth + sg.depth_off, m.Nnu,
                                   m.bin_width, c2 ? m.data : nullptr, c2 ? m.err : nullptr,
                                   binned + sg.bin_off, c2 ? c2 + sg.first : nullptr);
                BM_CHECK_HIP(hipGetLastError());
            }
        }
    }
    return BM_OK;
}

// ---- tuned configurations --------------------------------------------------------------
// Keyed by the batch signature: dtype, species count, CIA, and every run of samples
// (instance shape and count) in order.
static std::string batch_signature(const bm_model* models, const HostPlan& hp) {
    std::string s = std::to_string(models[0].dtype) + ":" + std::to_string(hp.n_species) + ":" +
                    std::to_string((int)hp.cia);
    for (const LaunchPlan& lp : hp.plans)
        for (int i = 0; i < lp.n_seg; ++i) {
            const Segment& sg = lp.seg[i];
            const ModelDev& m = lp.model[sg.model];
            s += "|" + std::to_string(m.L) + "x" + std::to_string(m.Nnu) + "x" + std::to_string(m.NT) + "x" +
                 std::to_string(m.NTc) + "b" + std::to_string(m.bin_width) + "n" + std::to_string(sg.count);
        }
    return s;
}

static std::mutex g_tune_mu;
static std::map<std::string, int>* g_tuned = nullptr;

// Untuned batches: cached table loads; chord weights staged in LDS while the launch has
// at most two workgroups per CU (one or a few spectra), streamed from L2 beyond that (LDS
// would then cap the workgroups per CU). Measured on MI355X for the config-2 shapes.
static int default_config(const HostPlan& hp) {
    size_t wgs = 0;
    for (const LaunchPlan& lp : hp.plans) wgs += (size_t)lp.total_wgs;
    return wgs <= 2 * 256 ? 1 : 3;
}

static int tuned_config(const bm_model* models, const HostPlan& hp) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    if (!g_tuned || g_tuned->empty()) return default_config(hp);
    auto it = g_tuned->find(batch_signature(models, hp));
    return it == g_tuned->end() ? default_config(hp) : it->second;
}

static int run_forward(const bm_model* models, const HostPlan& hp, int cfg, const double* params, int stride,
                       const int32_t* active, double* depth, double* binned, double* chi2, int32_t* flags,
                       void* ws, hipStream_t s) {
    if (models[0].dtype == BM_F32)
        return launch_forward<float>(hp, cfg, params, stride, active, depth, binned, chi2, flags, (char*)ws, s);
    return launch_forward<double>(hp, cfg, params, stride, active, depth, binned, chi2, flags, (char*)ws, s);
}

// argument checks shared by bm_forward_batch and bm_forward_tune
static int check_forward_args(const bm_model* models, int n_models, const int32_t* instance, const double* params,
                              int param_stride, int B, double* depth, double* binned, double* chi2,
                              int32_t* flags, void* workspace, size_t workspace_bytes, HostPlan& hp) {
    if (!models || !params || !depth || !flags || !workspace) return BM_EINVAL;
    int st = build_plans(models, n_models, instance, B, hp);
    if (st != BM_OK) return st;
    for (int i = 0; i < n_models; ++i) {
        if (param_stride < bm_n_params(&models[i])) return BM_ESHAPE;
        if (binned && models[i].bin_width <= 0) return BM_EINVAL;
        if (chi2 && (!models[i].data || !models[i].err)) return BM_EINVAL;
    }
    if (chi2 && !binned) return BM_EINVAL;
    if (workspace_bytes < hp.ws_bytes) return BM_ENOSPACE;
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
        case BM_ESCRATCH: return "request needs more than the no-allocation scratch array (BM_NOALLOC_SCRATCH_BYTES)";
        default: return "unknown status";
    }
}

extern "C" int bm_version(void) { return 102; }

extern "C" size_t bm_struct_size(int which) {
    switch (which) {
        case 0: return sizeof(bm_planet);
        case 1: return sizeof(bm_model);
        case 2: return sizeof(bm_demcz);
        case 3: return sizeof(bm_mlp);
        case 4: return sizeof(bm_voigt_grid);
        default: return 0;
    }
}

extern "C" int bm_n_params(const bm_model* model) {
    if (!model) return BM_EINVAL;
    return (model->tp_mode == BM_TP_ISOTHERMAL ? 1 : 5) + model->n_species + 1 + (model->cloud ? 1 : 0);
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

namespace bm {
__global__ void k_cia_combine(const double* __restrict__ a, const double* __restrict__ b, double r, int64_t n,
                              double* out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a[i] + r * b[i];
}
}  // namespace bm

extern "C" int bm_cia_combine(const double* k_h2h2, const double* k_h2he, double ratio, int64_t n, double* out,
                              void* stream) {
    using namespace bm;
    if (n < 0) return BM_ESHAPE;
    if (n == 0) return BM_OK;
    if (!k_h2h2 || !k_h2he || !out || !std::isfinite(ratio) || ratio < 0.0) return BM_EINVAL;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_cia_combine, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, k_h2h2, k_h2he,
                       ratio, n, out);
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

extern "C" size_t bm_sigma_tiles_bytes(const bm_model* model, int tile_w) {
    if (!model || validate_model(*model, true) != BM_OK || tile_w < 1 || tile_w > kTileNu) return 0;
    return sigma_tiles_bytes(*model, tile_w);
}

extern "C" int bm_sigma_tiles(const bm_model* model, int tile_w, void* out, size_t out_bytes, void* stream) {
    if (!model || !out) return BM_EINVAL;
    const int v = validate_model(*model, true);
    if (v != BM_OK) return v;
    if (tile_w < 1 || tile_w > kTileNu) return BM_EINVAL;
    const size_t need = sigma_tiles_bytes(*model, tile_w);
    if (out_bytes < need) return BM_ENOSPACE;
    const int n_tiles = (model->n_nu + tile_w - 1) / tile_w;
    const size_t n_rows = (size_t)model->n_species * model->n_temp;
    const size_t total = n_rows * (size_t)n_tiles * model->n_layers * tile_w;
    const unsigned grid = (unsigned)std::min<size_t>((total + 255) / 256, 1u << 16);
    hipStream_t st = (hipStream_t)stream;
    if (model->dtype == BM_F32)
        hipLaunchKernelGGL(k_sigma_tiles<float>, dim3(grid), dim3(256), 0, st, static_cast<const float*>(model->sigma),
                           model->n_layers, model->n_nu, tile_w, n_tiles, n_rows, static_cast<float*>(out));
    else
        hipLaunchKernelGGL(k_sigma_tiles<double>, dim3(grid), dim3(256), 0, st, static_cast<const double*>(model->sigma),
                           model->n_layers, model->n_nu, tile_w, n_tiles, n_rows, static_cast<double*>(out));
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

extern "C" int bm_forward_batch(const bm_model* models, int n_models, const int32_t* instance,
                                const double* params, int param_stride, int B, const int32_t* active,
                                double* depth, double* binned, double* chi2, int32_t* flags, void* workspace,
                                size_t workspace_bytes, void* stream) {
    HostPlan hp;
    int st = check_forward_args(models, n_models, instance, params, param_stride, B, depth, binned, chi2, flags,
                                workspace, workspace_bytes, hp);
    if (st != BM_OK) return st;
    if (B == 0) return BM_OK;
    const int cfg = tuned_config(models, hp);
    return run_forward(models, hp, cfg, params, param_stride, active, depth, binned, chi2, flags, workspace,
                       (hipStream_t)stream);
}

// ---- no-allocation form ----------------------------------------------------------------
// The per-sample records and the list of requested samples live in a fixed device array
// instead of a caller workspace. Host code never passes the array's name to a kernel (on
// the host it is a stand-in, not a device address): its address on each device is looked
// up once, with that device current, and kept.
static __device__ __align__(256) char scratch[BM_NOALLOC_SCRATCH_BYTES];

static int scratch_address(void** out) {
    constexpr int kMaxDevices = 64;
    static void* per_device[kMaxDevices] = {nullptr};
    static std::mutex mu;
    int dev = 0;
    BM_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return BM_EHIP;
    std::lock_guard<std::mutex> lock(mu);
    if (!per_device[dev]) {
        void* p = nullptr;
        BM_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return BM_EHIP;
        per_device[dev] = p;
    }
    *out = per_device[dev];
    return BM_OK;
}

extern "C" int bm_forward_batch_noalloc(const bm_model* models, int n_models, const int32_t* instance,
                                        const double* params, int param_stride, int B, const int32_t* active,
                                        double* depth, double* binned, double* chi2, int32_t* flags,
                                        void* stream) {
    // the size check runs before any device call: a request beyond the array fails at once
    {
        HostPlan probe;
        const int st = build_plans(models, n_models, instance, B, probe);
        if (st != BM_OK) return st;
        if (probe.ws_bytes > (size_t)BM_NOALLOC_SCRATCH_BYTES) return BM_ESCRATCH;
    }
    HostPlan hp;
    int st;
    void* ws = nullptr;
    st = scratch_address(&ws);
    if (st != BM_OK) return st;
    st = check_forward_args(models, n_models, instance, params, param_stride, B, depth, binned, chi2, flags, ws,
                            (size_t)BM_NOALLOC_SCRATCH_BYTES, hp);
    if (st != BM_OK) return st;
    if (B == 0) return BM_OK;
    const int cfg = tuned_config(models, hp);
    return run_forward(models, hp, cfg, params, param_stride, active, depth, binned, chi2, flags, ws,
                       (hipStream_t)stream);
}

extern "C" int bm_forward_config_count(void) { return kNumFwdConfigs; }

extern "C" const char* bm_forward_config_name(int config) {
    if (config < 0 || config >= kNumFwdConfigs) return nullptr;
    return kFwdConfigs[config].name;
}

extern "C" int bm_forward_tune(const bm_model* models, int n_models, const int32_t* instance, const double* params,
                               int param_stride, int B, double* depth, double* binned, double* chi2, int32_t* flags,
                               void* workspace, size_t workspace_bytes, void* stream, int reps, int* chosen,
                               float* times_ms, int n_times) {
    HostPlan hp;
    int st = check_forward_args(models, n_models, instance, params, param_stride, B, depth, binned, chi2, flags,
                                workspace, workspace_bytes, hp);
    if (st != BM_OK) return st;
    if (reps < 1 || B < 1) return BM_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    BM_CHECK_HIP(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) return BM_EINVAL;
    const int n_cfg = models[0].dtype == BM_F32 ? kNumFwdConfigs : 1;
    hipEvent_t e0, e1;
    BM_CHECK_HIP(hipEventCreate(&e0));
    BM_CHECK_HIP(hipEventCreate(&e1));
    int best = 0;
    float best_ms = 0.f;
    int code = BM_OK;
    for (int c = 0; c < kNumFwdConfigs && code == BM_OK; ++c) {
        float ms = -1.f;
        if (c < n_cfg) {
            code = run_forward(models, hp, c, params, param_stride, nullptr, depth, binned, chi2, flags, workspace, s);
            if (code == BM_ESHAPE) {  // this configuration does not fit the batch (LDS)
                code = BM_OK;
            } else if (code == BM_OK) {
                if (hipEventRecord(e0, s) != hipSuccess) code = BM_EHIP;
                for (int r = 0; r < reps && code == BM_OK; ++r)
                    code = run_forward(models, hp, c, params, param_stride, nullptr, depth, binned, chi2, flags,
                                       workspace, s);
                if (code == BM_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                      hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    code = BM_EHIP;
                if (code == BM_OK) {
                    ms /= reps;
                    if (best_ms == 0.f || ms < best_ms) {
                        best_ms = ms;
                        best = c;
                    }
                }
            }
        }
        if (times_ms && c < n_times) times_ms[c] = ms;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (code != BM_OK) return code;
    if (best_ms == 0.f) return BM_ESHAPE;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        if (!g_tuned) g_tuned = new std::map<std::string, int>();
        (*g_tuned)[batch_signature(models, hp)] = best;
    }
    if (chosen) *chosen = best;
    return BM_OK;
}

extern "C" int bm_forward_set_config(const bm_model* models, int n_models, const int32_t* instance, int B,
                                     int config) {
    if (config < -1 || config >= kNumFwdConfigs) return BM_EINVAL;
    HostPlan hp;
    int st = build_plans(models, n_models, instance, B, hp);
    if (st != BM_OK) return st;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    if (!g_tuned) g_tuned = new std::map<std::string, int>();
    if (config < 0)
        g_tuned->erase(batch_signature(models, hp));
    else
        (*g_tuned)[batch_signature(models, hp)] = config;
    return BM_OK;
}

extern "C" int bm_timing_start(int capacity) {
    if (capacity < 1 || capacity > (1 << 20)) return BM_EINVAL;
    std::lock_guard<std::mutex> lock(g_timing_mu);
    if (g_timing) return BM_EINVAL;
    TimingSession* t = new TimingSession();
    t->ev.resize(2 * (size_t)capacity, nullptr);
    for (auto& e : t->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto& f : t->ev)
                if (f) hipEventDestroy(f);
            delete t;
            return BM_EHIP;
        }
    }
    t->cap = capacity;
    g_timing = t;
    return BM_OK;
}

extern "C" int bm_timing_stop(double* total_ms, int64_t* launches) {
    TimingSession* t;
    {
        std::lock_guard<std::mutex> lock(g_timing_mu);
        t = g_timing;
        g_timing = nullptr;
    }
    if (!t) return BM_EINVAL;
    double tot = 0.0;
    int code = BM_OK;
    for (int i = 0; i < t->used; ++i) {
        float ms = 0.f;
        if (hipEventSynchronize(t->ev[2 * i + 1]) != hipSuccess ||
            hipEventElapsedTime(&ms, t->ev[2 * i], t->ev[2 * i + 1]) != hipSuccess) {
            code = BM_EHIP;
            break;
        }
        tot += ms;
    }
    const int used = t->used;
    for (auto& e : t->ev) hipEventDestroy(e);
    delete t;
    if (total_ms) *total_ms = tot;
    if (launches) *launches = used;
    return code;
}
