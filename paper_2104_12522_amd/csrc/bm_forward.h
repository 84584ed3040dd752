// Shared declarations of the forward-model kernels (internal).
#pragma once
#include <cstddef>

#include <vector>

#include "bm_internal.h"

namespace bm {

constexpr int kAtmThreads = BM_MAX_LAYERS;  // threads for one-sample atmosphere work (>= L)
constexpr int kRows = 8;                    // chord-weight rows per register block (FP64 path)
constexpr int kTileNu = kWave;              // wavenumbers per forward workgroup (one per lane)
constexpr int kMaxModels = 4;               // distinct models in one fused launch
constexpr int kMaxSegments = 16;            // runs of same-model samples in one launch

// FP32 chord contraction on the matrix cores: v_mfma_f32_16x16x4f32 multiplies a 16x4
// block of chord weights (rows j, layers l) by a 4x16 block of extinction (layers l,
// wavenumbers). Row block J holds rows [16J, 16J+16) and runs over layers [16J, L).
// The k-steps of a row block are padded with zero weights to a multiple of kMfmaChunk.
constexpr int kMfmaM = 16;
constexpr int kMfmaK = 4;
constexpr int kMfmaChunk = 4;

__host__ __device__ inline int mfma_row_blocks(int L) { return (L - 1 + kMfmaM - 1) / kMfmaM; }
__host__ __device__ inline int mfma_ksteps(int L, int J) {
    const int raw = (L - kMfmaM * J + kMfmaK - 1) / kMfmaK;
    return (raw + kMfmaChunk - 1) / kMfmaChunk * kMfmaChunk;
}
// sum of the k-steps of row blocks 0..J-1: mfma_ksteps(L, i) = 4 (ceil(L/16) - i)
__host__ __device__ inline int mfma_kstep_offset(int L, int J) {
    const int c = (L + kMfmaM - 1) / kMfmaM;
    return kMfmaChunk * (J * c - J * (J - 1) / 2);
}
__host__ __device__ inline int mfma_total_ksteps(int L) { return mfma_kstep_offset(L, mfma_row_blocks(L)); }

// broadcast lane `i` (uniform) of a per-lane value to the whole wave (v_readlane)
__device__ __forceinline__ int lane_get(int v, int i) { return __builtin_amdgcn_readlane(v, i); }
__device__ __forceinline__ float lane_get(float v, int i) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), i));
}
__device__ __forceinline__ double lane_get(double v, int i) {
    const long long u = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), i);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), i);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Device view of a bm_model (passed by value in kernel arguments).
struct ModelDev {
    const void* sigma;
    const void* sigma_tiles;  // tile-major copy [S][NT][tiles][L][64] for tile width tile_w, or null
    const double* temp;
    const double* cia;
    const double* temp_cia;
    const double* p_bar;
    const double* data;
    const double* err;
    int S, NT, L, Nnu, NTc, tp_mode, bin_width, nb;
    int rayleigh, cloud, geometry;
    int tile_w;  // tile width of sigma_tiles
    double mass[BM_MAX_SPECIES];
    bm_planet pl;
    double tau_max;  // optical-depth limit (+infinity: none)
    double nu_start, dnu;
};

// A run of consecutive samples that use the same model.
struct Segment {
    int model;
    int first;           // first sample index (relative to the launch)
    int count;           // samples in the run
    int tiles;           // wavenumber tiles per sample
    int tile_begin;      // first workgroup index of the run
    int tiles_per_xcd;   // tiles owned by each XCD (tile-major, XCD-aware order)
    int tile_w;          // wavenumbers per tile (a whole number of channels when binning)
    int fused_bins;      // 1: each tile bins its own channels; 0: no binning in the kernel
    size_t ws_off;       // byte offset of the run's first record in the workspace
    size_t rec_bytes;    // bytes per sample record
    size_t depth_off;    // offset (elements) of the run's first spectrum in `depth`
    size_t bin_off;      // offset (elements) of the run's first binned spectrum
};

struct LaunchPlan {
    ModelDev model[kMaxModels];
    Segment seg[kMaxSegments];
    int n_seg;
    int total_wgs;
    int max_ntc;   // largest CIA temperature grid among the models (LDS staging rows)
    int prio_from; // pipelined launches: first workgroup of the second dispatch round, when the
                   // launch has at most two rounds (set at launch; else no workgroup qualifies)
    __device__ int segment_of_sample(int b) const {
        int s = 0;
        for (int i = 1; i < n_seg; ++i)
            if (b >= seg[i].first) s = i;
        return s;
    }
    __device__ int segment_of_wg(int t) const {
        int s = 0;
        for (int i = 1; i < n_seg; ++i)
            if (t >= seg[i].tile_begin) s = i;
        return s;
    }
};

// Workgroups of a segment: count * 8 * tiles_per_xcd. Workgroup g (local index) runs on
// XCD g % 8 (round-robin dispatch); the k-th workgroup of an XCD takes tile
// xcd * tiles_per_xcd + k / count of sample k % count, so each XCD sweeps a contiguous
// wavenumber range and all samples of one tile run back to back on the same L2.
constexpr int kXcds = 8;
__host__ __device__ inline int segment_wgs(int count, int tiles) {
    return count * kXcds * ((tiles + kXcds - 1) / kXcds);
}

struct RecordHeader {
    double base;     // r_0^2
    double rs2;      // stellar radius squared
    int32_t flags;   // sample flags
    int32_t counter; // unused
    int32_t jcloud;  // chords j <= jcloud lie in or below the cloud deck (-1: none)
    int32_t pad;
};
// the fused kernel reads flags .. pad as int32 words 4 .. 7 of the header
static_assert(offsetof(RecordHeader, flags) == 16 && offsetof(RecordHeader, jcloud) == 24 &&
                  sizeof(RecordHeader) == 32, "record header layout");

inline __host__ __device__ size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline __host__ __device__ int row_blocks(int L) { return (L + kRows - 1) / kRows; }

// chord-weight entries of one sample: MFMA A fragments (FP32) or 8-row blocks (FP64)
template <typename T>
__host__ __device__ inline size_t chord_weight_entries(int L) {
    if (sizeof(T) == 4) return (size_t)mfma_total_ksteps(L) * kWave;
    return (size_t)row_blocks(L) * L * kRows;
}

// Byte layout of one sample record for compute type T.
template <typename T>
struct RecordLayout {
    size_t hdr, kidx, kcidx, w, wc, bfac, rfac, afac, cw, tl, rl, wb, total;
    __host__ __device__ RecordLayout(int S, int L) {
        size_t o = 0;
        hdr = o;   o = align_up(o + sizeof(RecordHeader), 64);
        kidx = o;  o = align_up(o + sizeof(int32_t) * L, 64);
        kcidx = o; o = align_up(o + sizeof(int32_t) * L, 64);
        w = o;     o = align_up(o + sizeof(T) * L, 64);
        wc = o;    o = align_up(o + sizeof(double) * L, 64);
        bfac = o;  o = align_up(o + sizeof(double) * L, 64);
        rfac = o;  o = align_up(o + sizeof(T) * L, 64);
        afac = o;  o = align_up(o + sizeof(T) * L * S, 64);
        cw = o;    o = align_up(o + sizeof(double) * L, 64);
        tl = o;    o = align_up(o + sizeof(double) * L, 64);
        rl = o;    o = align_up(o + sizeof(double) * L, 64);
        wb = o;    o = align_up(o + sizeof(T) * chord_weight_entries<T>(L), 256);
        total = o;
    }
};

template <typename T>
struct RecordView {
    RecordHeader* hdr;
    int32_t* kidx;
    int32_t* kcidx;
    T* w;
    double* wc;    // CIA interpolation weight
    double* bfac;  // n_H2^2 (overflows float: the CIA term is formed in double)
    T* rfac;       // n_H2 (Rayleigh scattering)
    T* afac;       // [S][L] absorber number densities
    double* cw;    // impact-parameter weight of f_j
    double* tl;    // layer temperatures (emission source)
    double* rl;    // layer radii (emission path lengths)
    T* wb;         // chord weights (layout: chord_weight_entries)
    double* chi2part;  // [tiles] chi^2 of each tile's channels (after the fixed layout)
    __host__ __device__ RecordView(char* base, int S, int L) {
        RecordLayout<T> lay(S, L);
        hdr = (RecordHeader*)(base + lay.hdr);
        kidx = (int32_t*)(base + lay.kidx);
        kcidx = (int32_t*)(base + lay.kcidx);
        w = (T*)(base + lay.w);
        wc = (double*)(base + lay.wc);
        bfac = (double*)(base + lay.bfac);
        rfac = (T*)(base + lay.rfac);
        afac = (T*)(base + lay.afac);
        cw = (double*)(base + lay.cw);
        tl = (double*)(base + lay.tl);
        rl = (double*)(base + lay.rl);
        wb = (T*)(base + lay.wb);
        chi2part = (double*)(base + lay.total);
    }
};

// bytes of one sample record including the per-tile chi^2 partials
template <typename T>
__host__ __device__ inline size_t record_bytes_t(int S, int L, int tiles) {
    return RecordLayout<T>(S, L).total + align_up(sizeof(double) * (size_t)tiles, 256);
}

// host helpers (forward.hip)
int validate_model(const bm_model& m, bool need_tables);
ModelDev to_device_view(const bm_model& m);
// compute units of the current device (cached per device; 0 if unknown)
int device_cu_count();
// raise a kernel's dynamic-LDS ceiling (once per kernel, device and size)
int ensure_dynamic_lds(const void* fn, size_t bytes);

// A batch split into launch plans of at most kMaxSegments same-model runs each.
struct HostPlan {
    std::vector<LaunchPlan> plans;
    std::vector<int> first_sample;   // first sample of each plan
    std::vector<int> n_samples;      // samples of each plan
    size_t ws_bytes = 0;
    size_t list_off = 0;      // workspace offset of the requested-sample list (B + 1 int32)
    int max_L = 0;
    int n_species = 0;
    bool cia = false;
    int max_ntc = 0;          // largest CIA temperature grid (LDS staging rows)
    int geometry = 0;         // BM_GEOM_TRANSIT or BM_GEOM_ECLIPSE (all models of a batch)
    int total_samples = 0;
    size_t max_entries = 0;   // chord-weight entries of the largest record
};

// emission geometry: intensity of samples [first, first + count) of one segment
template <typename T>
int launch_k_emission(const LaunchPlan& lp, int seg, char* ws, const int32_t* act, double* out, hipStream_t st);

// launch of the fused kernel for one plan with kW waves per workgroup, non-temporal (kNT)
// or cached table loads, and phase-2 mode kMode (chord weights streamed from L2, staged in
// LDS, or staged with phases 1 and 2 interleaved; fwd_kernel.h); compact (or null) is the
// list of requested samples of a masked call and compact_count its length, run in
// compact_slots sample slots per tile; ev0/ev1 (or null) are timing events that the
// dispatch itself records at the kernel's start and end
template <typename T, int kW, bool kNT, int kMode>
int launch_k_forward(const HostPlan& hp, const LaunchPlan& lp, size_t lds, char* ws, const int32_t* act,
                     double* depth, double* binned, double* c2, const int32_t* compact,
                     const int32_t* compact_count, int compact_slots, hipStream_t st, hipEvent_t ev0,
                     hipEvent_t ev1);

// record preparation; kSingle: a single-segment plan whose model is in slot 0;
// kMasked: `active` is not null; compact (or null): the list of requested samples of a
// masked call and compact_count its length, taken in turn by gridDim.x sample slots;
// build_n > 0: the kernel builds that list itself from the build_n flags of `active` (at most
// kPrepListMax) and writes it to compact, its length to compact[build_n]
constexpr int kPrepListMax = 1024;
template <typename T, bool kSingle, bool kMasked>
__global__ void k_atm_prep(LaunchPlan plan, const double* __restrict__ params, int stride,
                           const int32_t* __restrict__ active, char* __restrict__ ws,
                           int32_t* __restrict__ flags_out, int32_t* __restrict__ compact,
                           const int32_t* __restrict__ compact_count, int build_n);

}  // namespace bm
