// Shared declarations of the forward-model kernels (internal).
#pragma once

#include "bm_internal.h"

namespace bm {

constexpr int kAtmThreads = BM_MAX_LAYERS;  // one thread per layer in the atmosphere kernels
constexpr int kRows = 8;                    // chord-weight rows per register block
constexpr int kTileNu = kWave;              // wavenumbers per forward workgroup (one per lane)
constexpr int kMaxModels = 4;               // distinct models in one fused launch
constexpr int kMaxSegments = 16;            // runs of same-model samples in one launch

// Device view of a bm_model (passed by value in kernel arguments).
struct ModelDev {
    const void* sigma;
    const double* temp;
    const void* cia;
    const double* temp_cia;
    const double* p_bar;
    const double* data;
    const double* err;
    int S, NT, L, Nnu, NTc, tp_mode, bin_width, nb;
    double mass[BM_MAX_SPECIES];
    bm_planet pl;
};

// A run of consecutive samples that use the same model.
struct Segment {
    int model;
    int first;           // first sample index
    int count;           // samples in the run
    int tiles;           // wavenumber tiles per sample
    int tile_begin;      // first global tile index of the run
    int pad;
    size_t ws_off;       // byte offset of the run's first record in the workspace
    size_t rec_bytes;    // bytes per sample record
    size_t depth_off;    // offset (elements) of the run's first spectrum in `depth`
    size_t bin_off;      // offset (elements) of the run's first binned spectrum
};

struct LaunchPlan {
    ModelDev model[kMaxModels];
    Segment seg[kMaxSegments];
    int n_seg;
    int total_tiles;
    __device__ int segment_of_sample(int b) const {
        int s = 0;
        for (int i = 1; i < n_seg; ++i)
            if (b >= seg[i].first) s = i;
        return s;
    }
    __device__ int segment_of_tile(int t) const {
        int s = 0;
        for (int i = 1; i < n_seg; ++i)
            if (t >= seg[i].tile_begin) s = i;
        return s;
    }
};

struct RecordHeader {
    double base;     // r_0^2
    double rs2;      // stellar radius squared
    int32_t flags;   // sample flags
    int32_t counter; // tiles finished (reset to zero by the last tile)
    int32_t pad[2];
};

inline __host__ __device__ size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline __host__ __device__ int row_blocks(int L) { return (L + kRows - 1) / kRows; }

// Byte layout of one sample record for compute type T.
template <typename T>
struct RecordLayout {
    size_t hdr, kidx, kcidx, w, wc, bfac, afac, cw, wb, total;
    __host__ __device__ RecordLayout(int S, int L) {
        size_t o = 0;
        hdr = o;   o = align_up(o + sizeof(RecordHeader), 64);
        kidx = o;  o = align_up(o + sizeof(int32_t) * L, 64);
        kcidx = o; o = align_up(o + sizeof(int32_t) * L, 64);
        w = o;     o = align_up(o + sizeof(T) * L, 64);
        wc = o;    o = align_up(o + sizeof(T) * L, 64);
        bfac = o;  o = align_up(o + sizeof(T) * L, 64);
        afac = o;  o = align_up(o + sizeof(T) * L * S, 64);
        cw = o;    o = align_up(o + sizeof(double) * L, 64);
        wb = o;    o = align_up(o + sizeof(T) * (size_t)row_blocks(L) * L * kRows, 256);
        total = o;
    }
};

template <typename T>
struct RecordView {
    RecordHeader* hdr;
    int32_t* kidx;
    int32_t* kcidx;
    T* w;
    T* wc;
    T* bfac;
    T* afac;   // [S][L]
    double* cw;
    T* wb;     // [nb][L][kRows]
    int nb;
    __host__ __device__ RecordView(char* base, int S, int L) {
        RecordLayout<T> lay(S, L);
        hdr = (RecordHeader*)(base + lay.hdr);
        kidx = (int32_t*)(base + lay.kidx);
        kcidx = (int32_t*)(base + lay.kcidx);
        w = (T*)(base + lay.w);
        wc = (T*)(base + lay.wc);
        bfac = (T*)(base + lay.bfac);
        afac = (T*)(base + lay.afac);
        cw = (double*)(base + lay.cw);
        wb = (T*)(base + lay.wb);
        nb = row_blocks(L);
    }
};

// host helpers (forward.hip)
int validate_model(const bm_model& m, bool need_tables);
ModelDev to_device_view(const bm_model& m);

template <typename T>
__global__ void k_atm_prep(LaunchPlan plan, const double* __restrict__ params, int stride,
                           char* __restrict__ ws, int32_t* __restrict__ flags_out);

}  // namespace bm
