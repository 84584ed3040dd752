// Steps a3-a6 of the forward model on the GPU and the C-ABI entry points that expose
// them: temperature interpolation of the opacity tables and extinction (Sec. 3,
// Sec. 6.1.1), chord optical depth through spherical layers and the transit-depth
// integral over impact parameter (Sec. 6.1), channel binning and chi^2 (Sec. 3).
//
// Hot kernel: k_forward. One workgroup (8 waves) owns one tile of up to 64 consecutive
// wavenumbers (one per lane; a whole number of channels when binning) of one sample:
//   phase 1  extinction. Wave w owns a contiguous run of layers; their record fields
//            (T bracket, weights, densities) sit one layer per lane and are broadcast
//            with v_readlane, so the two bracketing temperature rows of every species
//            table are streamed for four layers at a time (coalesced along
//            wavenumber, non-temporal or cached) with no memory wait for addresses, from
//            the tile-major copy of the tables when one exists for the tile width. CIA
//            rows of the tile are staged in LDS once. e[l][nu] is left in LDS.
//   (pipelined mode: phases 1 and 2 interleaved over 16-layer stages, see below)
//   phase 2  chord optical depth on the matrix cores (FP32): v_mfma_f32_16x16x4f32 over
//            16-row blocks of the triangular chord-weight matrix (A, staged in LDS) and
//            4-layer slices of e (B); items (row block, 16-column group) are dealt to
//            waves in snake order. Each finished optical depth becomes 1 - exp(-tau) and
//            is accumulated in double with its impact-parameter weight; partial sums are
//            combined in a fixed order. FP64 uses the vector ALU with 8-row blocks.
//   phase 3  the tile bins its own channels and writes its chi^2 partial; a small
//            kernel sums the partials per sample in a fixed tree.
// Workgroups are ordered XCD-aware and tile-major (see Segment) so that, in a batch,
// all samples of one tile read the same table rows from the same L2. A masked call of one
// run of samples can launch over the device-built list of its requested samples instead
// (the compacted variant).
#pragma once
#include <hip/hip_ext.h>
#include <climits>
#include <type_traits>

#include "bm_forward.h"

namespace bm {

template <typename T, bool kNonTemporal>
__device__ __forceinline__ T ld_table(const T* p) {
    if constexpr (kNonTemporal)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

// LDS layout of one forward workgroup (bytes from the start of dynamic shared memory):
//   es    extinction tile [rows][64] (FP32: L rounded up to 4 plus 16 zero rows, the
//         furthest a padded k-step reaches; pipelined: L rounded up to 16)
//   cw    impact-parameter weights [L] (double)
//   u     CIA rows of the tile [NTc][64] (double) during phase 1; afterwards the
//         per-row-block partial sums [blocks][64] and the tile's depths [64] (pipelined:
//         separate regions, since row blocks finish while CIA rows are still read), and
//         in FP64 after those the waves' chord-weight chunks [waves][kChunkL][8] (double)
// Staged configurations keep the sample's FP32 chord-weight fragments in a static LDS
// array, copied from the record straight into LDS at kernel start; it holds the fragments
// of up to kStageMaxLayers layers (36 KB), or kPipeMaxLayers (28 KB) when pipelined.
constexpr int kStageMaxLayers = 128;
constexpr int kStageMaxFloats = 144 * kWave;  // mfma_total_ksteps(128) k-steps of 64 lanes
constexpr int kPipeMaxLayers = 112;
constexpr int kPipeMaxFloats = 112 * kWave;   // mfma_total_ksteps(112)

// launch modes of the fused kernel's FP32 phase 2
constexpr int kModeStreamed = 0;   // chord weights read from L2 in phase 2
constexpr int kModeStaged = 1;     // chord weights in LDS, phase 2 after phase 1
constexpr int kModePipelined = 2;  // chord weights in LDS, phases 1 and 2 interleaved by stage

template <int kMode>
struct StageSize {
    static constexpr int floats = kMode == kModeStaged ? kStageMaxFloats : (kMode == kModePipelined ? kPipeMaxFloats : 0);
    static constexpr int chunks = floats / (4 * kWave);      // 16-byte-per-lane copies
    static constexpr int chunks_per_wave = (chunks + 7) / 8;  // 8 waves per workgroup
};

// FP64 chord sums: each wave streams its row block's chord weights through a private LDS
// chunk of kChunkL layers (32 layers x 8 rows x 8 bytes = 2 KB, two 16-byte pieces per lane)
constexpr int kChunkL = 32;

template <typename T>
struct FwdLds {
    size_t es, cw, ciat, part, bins, wst, total;
    int es_rows;
    __host__ __device__ FwdLds(int L, int kWaves, int ntc, bool pipe = false) {
        if (sizeof(T) == 4)
            es_rows = pipe ? kMfmaM * ((L + kMfmaM - 1) / kMfmaM) : ((L + 3) & ~3) + kMfmaM;
        else
            es_rows = L;
        es = 0;
        size_t o = align_up(sizeof(T) * (size_t)es_rows * kTileNu, 16);
        cw = o;
        o = align_up(o + sizeof(double) * (size_t)L, 16);
        ciat = o;
        const int nparts = (sizeof(T) == 4) ? mfma_row_blocks(L) : kWaves;
        size_t u1 = sizeof(double) * (size_t)ntc * kTileNu;
        if (pipe) {
            part = align_up(o + u1, 16);
            bins = part + sizeof(double) * (size_t)nparts * kTileNu;
            o = bins + sizeof(double) * kTileNu;
        } else {
            part = o;
            bins = part + sizeof(double) * (size_t)nparts * kTileNu;
            const size_t u2 = bins + sizeof(double) * kTileNu - o;
            // FP64: the waves' chord-weight chunks follow the partial sums and bins, over
            // the CIA rows' tail (the CIA rows are dead after phase 1, which a barrier
            // closes; the partial sums and bins are written while other waves still read
            // their chunks, so they stay apart)
            wst = align_up(bins + sizeof(double) * kTileNu, 16);
            size_t u = u1 > u2 ? u1 : u2;
            if (sizeof(T) == 8) {
                const size_t u3 = wst + sizeof(double) * (size_t)kWaves * kChunkL * kRows - o;
                if (u3 > u) u = u3;
            }
            o += u;
        }
        if (pipe) wst = o;  // unused (FP32 only)
        const size_t chi2_part = sizeof(double) * (size_t)kWaves * kWave;
        total = o > chi2_part ? o : chi2_part;
    }
};

// extinction tile element (l, column c): FP32 rows swap their 16-column halves on odd
// layers so that the matrix-core B reads (4 layers x 16 columns) are bank-conflict free
template <typename T>
__device__ __forceinline__ int es_index(int l, int c) {
    if constexpr (sizeof(T) == 4) return l * kTileNu + (c ^ ((l & 1) << 4));
    return l * kTileNu + c;
}


typedef __attribute__((address_space(3))) void* lds_void_ptr;

// absorbed fraction of a chord, 1 - exp(-tau), or 1 at and beyond the optical-depth limit
__device__ __forceinline__ double opaque_fraction(float tau, double tau_max) {
    return (double)tau >= tau_max ? 1.0 : (double)dev_absorbed(tau);
}
__device__ __forceinline__ double opaque_fraction(double tau, double tau_max) {
    return tau >= tau_max ? 1.0 : dev_absorbed(tau);
}
// chord j: opaque at and below the cloud deck's layer jcl, else as above
template <typename F>
__device__ __forceinline__ double chord_fraction(int j, int jcl, F tau, double tau_max) {
    return j <= jcl ? 1.0 : opaque_fraction(tau, tau_max);
}

// Record fields of the pipelined path, one layer per lane: lane i holds stage i / 2, layer
// Ltop - 16 (i / 2 + 1) + 2 wave + i % 2 (clamped to the model). The bracket indices are
// clamped into the tables, so that a record flagged for a failed radius solve still loads
// in bounds (its depth is set to NaN at the end).
template <typename T, int kS, bool kCia>
struct PipeFields {
    int k = 0, kc = 0;
    T w, rf, a[kS];
    double wc = 0.0, b = 0.0;
    __device__ __forceinline__ void load(const RecordView<T>& rec, int L, int Ltop, int wave, int lane,
                                         int nt, int ntc) {
        const int l = max(0, min(Ltop - kMfmaM * (lane / 2 + 1) + 2 * wave + (lane & 1), L - 1));
        k = min(max(rec.kidx[l], 0), nt - 2);
        w = rec.w[l];
        rf = rec.rfac[l];
#pragma unroll
        for (int i = 0; i < kS; ++i) a[i] = rec.afac[i * L + l];
        if constexpr (kCia) {
            kc = min(max(rec.kcidx[l], 0), ntc - 2);
            wc = rec.wc[l];
            b = rec.bfac[l];
        }
    }
};

// kSingle: the launch holds one run of samples whose model is in slot 0, so the segment and
// model fields sit at fixed argument offsets and are read without a dependent lookup
template <typename T, int kWaves, int kS, bool kCia, bool kNonTemporal, int kMode, bool kSingle = false,
          bool kCompact = false>
__global__ void __launch_bounds__(kWaves * kWave)
    k_forward(LaunchPlan plan, char* __restrict__ ws, const int32_t* __restrict__ active,
              double* __restrict__ depth, double* __restrict__ binned, double* __restrict__ chi2,
              const int32_t* __restrict__ compact, const int32_t* __restrict__ compact_count, int compact_slots) {
    constexpr bool kStageA = kMode != kModeStreamed;
    constexpr bool kPipe = kMode == kModePipelined;
    extern __shared__ __align__(16) char smem[];
    // staged chord-weight fragments: a separate LDS object, so that the compiler can tell
    // phase 1's LDS traffic from the in-flight copies and does not wait for them there
    __shared__ __align__(16) float wa_s[kStageA ? StageSize<kMode>::floats : 1];
    __shared__ __align__(16) float wa_dummy[kStageA ? 4 * kWave : 1];
    static_assert(!kStageA || (kWaves == 8 && sizeof(T) == 4), "staging is laid out for 8 FP32 waves");
    // A launch of at most two workgroups per CU has all of them resident from the start. The
    // second round's workgroups then start behind the first round's prologue loads on their
    // CU and finish about a fifth later; a higher wave priority through the prologue and the
    // first two stages lets them catch up (one spectrum per call: 27.7 -> 25.9 us, measured).
    const bool late_round = kPipe && (int)blockIdx.x >= plan.prio_from;
    if (late_round) __builtin_amdgcn_s_setprio(2);
    const int si = kSingle ? 0 : plan.segment_of_wg(blockIdx.x);
    const Segment& sg = plan.seg[si];
    const ModelDev& m = plan.model[kSingle ? 0 : sg.model];
    // XCD-aware order: workgroup g runs on XCD g % 8; each XCD sweeps its own contiguous
    // tile range and runs all samples of a tile back to back (shared table rows in L2).
    // A compacted launch (a masked call of one run of samples: compact lists the requested
    // samples, compact_count[0] of them) has compact_slots sample slots per tile, and
    // workgroup (tile, slot k) takes list entries k, k + slots, ... in turn, so that a call
    // that requests few samples launches few workgroups.
    // A compacted launch orders its workgroups slot-major (all tiles of slot 0, then slot 1,
    // ...): a call that requests few samples has its working workgroups dispatched first and
    // the idle slots' workgroups after them, instead of interleaved with them.
    const int slots = kCompact ? compact_slots : sg.count;
    const int g = blockIdx.x - sg.tile_begin;
    const int per_slot = kXcds * sg.tiles_per_xcd;
    const int gs = kCompact ? g % per_slot : g;
    const int kx = gs / kXcds;
    const int tile = (gs % kXcds) * sg.tiles_per_xcd + (kCompact ? kx : kx / slots);
    const int slot = kCompact ? g / per_slot : kx % slots;
    // The pipelined unmasked-list variant checks its exits (padding workgroup, sample not
    // requested) only after its first record loads are in flight: those loads are in bounds
    // for any workgroup, and the kernel-argument reads behind the checks then overlap them.
    constexpr bool kLateExit = kPipe && !kCompact;
    const bool pad = tile >= sg.tiles;  // padding workgroup of the XCD split
    if (!kLateExit && pad) return;
    // one sample of this workgroup's tile (the compacted variant runs it for each of its
    // list entries; the loop stays out of the other variants' code)
    auto run = [&](const int s_in) {
        const int b = sg.first + s_in;
        if (!kLateExit && active && !active[b]) return;  // sample not requested in this call
        const int L = m.L, Nnu = m.Nnu;
        const double tau_max = m.tau_max;
        const RecordView<T> rec(ws + sg.ws_off + (size_t)s_in * sg.rec_bytes, kS, L);
        const FwdLds<T> lay(L, kWaves, plan.max_ntc, kPipe);

        const int lane = threadIdx.x & (kWave - 1);
        // the wave index is uniform across a wave; readfirstlane lets the compiler keep the
        // layer loops and every per-layer record load on the scalar unit
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
        const int nu = tile * sg.tile_w + lane;
        const bool valid = lane < sg.tile_w && nu < Nnu;
        const int nu_c = valid ? nu : min(tile * sg.tile_w, Nnu - 1);

        // Table rows: row (species i, temperature k, layer l) of this lane's column sits at
        // tab + i s_stride + k t_stride + l l_stride. The tile-major copy (when built for this
        // tile width) holds the tile's rows as one contiguous block of tile_w-column rows, the
        // row-major tables as pieces of Nnu-long rows. Lanes past the tile reread its last
        // column (no extra lines fetched).
        const int tw = sg.tile_w;
        const bool tiled = m.sigma_tiles != nullptr && m.tile_w == tw;
        const T* __restrict__ tab = tiled ? static_cast<const T*>(m.sigma_tiles) + (size_t)tile * L * tw + min(lane, tw - 1)
                                          : static_cast<const T*>(m.sigma) + nu_c;
        const size_t l_stride = tiled ? (size_t)tw : (size_t)Nnu;
        const size_t t_stride = tiled ? (size_t)sg.tiles * L * tw : (size_t)L * Nnu;
        const size_t s_stride = (size_t)m.NT * t_stride;

        T* es = reinterpret_cast<T*>(smem + lay.es);
        double* part = reinterpret_cast<double*>(smem + lay.part);
        double* dsh = reinterpret_cast<double*>(smem + lay.bins);
        double* dout = depth + sg.depth_off + (size_t)s_in * Nnu;
        // record header: the pipelined path reads it with a vector load after its record
        // fields (a scalar load of this freshly written record would hold up every scalar
        // wait of the prologue until it returned)
        int flags = 0, jcl = -1;  // jcl: chords j <= jcl are opaque (cloud deck)
        if constexpr (!kPipe) {
            flags = rec.hdr->flags;
            jcl = m.cloud ? rec.hdr->jcloud : -1;
        }
        // this tile's channels (phase 3). The pipelined path works them out and fetches their
        // data and errors with its first loads, so that phase 3 does not wait on memory; the
        // other paths do it in phase 3 (their workgroups are short, and the scalar waits and
        // divisions in the prologue cost them up to 15 % at 256 samples per launch)
        int bw = 0, nbt = 0, nbins = 0, cg = 0;
        bool want_chi2 = false, own_bin = false;
        auto channels = [&]() {
            bw = m.bin_width;
            nbt = bw > 0 ? sg.tile_w / bw : 0;  // whole channels per tile
            nbins = bw > 0 ? Nnu / bw : 0;
            want_chi2 = (chi2 != nullptr) && m.data && m.err;
            cg = tile * nbt + lane;
            own_bin = binned != nullptr && sg.fused_bins && lane < nbt && cg < nbins;
        };
        if constexpr (kPipe) channels();
        double ch_data = 0.0, ch_err = 1.0;
        // this lane's H2 Rayleigh cross section (the record holds n_H2 per layer); zero without
        // Rayleigh scattering, so that the per-layer term needs no branch (a branch in the
        // extinction loop cost 16 % at 256 samples per launch)
        const T sray = m.rayleigh ? (T)rayleigh_h2_xsec(m.nu_start + m.dnu * nu_c) : T(0);
        double dval = __builtin_nan("");  // this lane's depth (wave 0)

        // The pipelined path does not wait for the header before its loads: a flagged sample
        // runs the same in-bounds loads and gets NaN depths at the end. Its record fields, on
        // which the first table addresses depend, are issued before the fragment copies (loads
        // return in issue order, so waiting for them does not wait for the copies).
        if (kPipe || !(flags & BM_FLAG_RADIUS)) {
            PipeFields<T, kS, kCia> pf;
            int hv = 0;  // header words flags, (unused), jcloud, pad in lanes 0-3 (pipelined)
            if constexpr (kPipe) {
                pf.load(rec, L, kPipeMaxLayers, wave, lane, m.NT, m.NTc);
                // header words 0-7 (base, rs2, flags, unused, jcloud, pad) in lanes 0-7
                hv = reinterpret_cast<const int32_t*>(rec.hdr)[lane & 7];
                if (want_chi2 && own_bin && wave == 0) {
                    ch_data = m.data[cg];
                    ch_err = m.err[cg];
                }
                if constexpr (kLateExit)
                    if (pad || (active && !active[b])) return;
            }
            // impact-parameter weights (read per optical depth in phase 2) and this tile's
            // columns of every CIA temperature row (read by many layers) go to LDS; all their
            // loads are issued before the first store
            double* cw_s = reinterpret_cast<double*>(smem + lay.cw);
            double* cia_s = reinterpret_cast<double*>(smem + lay.ciat);
            constexpr int kMaxPer = BM_MAX_TEMPS * kTileNu / (kWaves * kWave);
            double cv[kMaxPer];
            auto cia_load = [&]() {
                const int n = m.NTc * kTileNu;
    #pragma unroll
                for (int q = 0; q < kMaxPer; ++q) {
                    const int i = min((int)threadIdx.x + q * kWaves * kWave, n - 1);
                    const int col = min(tile * sg.tile_w + (i % kTileNu), Nnu - 1);
                    cv[q] = m.cia[(size_t)(i / kTileNu) * Nnu + col];
                }
            };
            auto cia_store = [&]() {
                const int n = m.NTc * kTileNu;
    #pragma unroll
                for (int q = 0; q < kMaxPer; ++q) {
                    const int i = threadIdx.x + q * kWaves * kWave;
                    if (i < n) cia_s[i] = cv[q];
                }
            };
            // pipelined path: these loads go before the fragment copies too, so that their LDS
            // stores (before the first barrier) do not wait for the copies
            double cwv = 0.0;
            if constexpr (kPipe) {
                static_assert(kPipeMaxLayers <= kWaves * kWave, "one impact-parameter weight per thread");
                cwv = rec.cw[min((int)threadIdx.x, L - 1)];
                if constexpr (kCia) cia_load();
            }
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (kStageA && sizeof(T) == 4) {
                // chord-weight fragments record -> LDS without passing through registers
                // (global_load_lds: lane i of a wave writes 16 bytes at dst + 16 i). Every wave
                // issues the same fixed number of copies, so the compiler's memory-counter waits
                // stay exact; copies past the sample's fragments reread chunk 0 into a dummy
                // LDS row. They overlap the prologue's loads and are complete at its barrier.
                const int n_chunks = mfma_total_ksteps(L) * kWave / (4 * kWave);  // <= StageSize::chunks
    #pragma unroll
                for (int i = 0; i < StageSize<kMode>::chunks_per_wave; ++i) {
                    const int q = wave + kWaves * i;
                    const bool real = q < n_chunks;
                    const float* src = rec.wb + (real ? q : 0) * 4 * kWave + 4 * lane;
                    float* dst = real ? wa_s + q * 4 * kWave : wa_dummy;
                    __builtin_amdgcn_global_load_lds((const void*)src, (lds_void_ptr)dst, 16, 0, 0);
                }
            }
            if constexpr (!kPipe) {
                for (int i = threadIdx.x; i < L; i += kWaves * kWave) cw_s[i] = rec.cw[i];
                if constexpr (kCia) {
                    cia_load();
                    cia_store();
                }
                __syncthreads();
            }

            if constexpr (kPipe) {
                // ---- phases 1 and 2 interleaved over stages of 16 layers, from the top ----------
                // Stage s holds layers [lo_s, lo_s + 16), lo_s = Ltop - 16 (s + 1).
                // Every row block J with 16 J <= lo_s takes one chunk (4 k-steps, the stage's
                // layers) from it, and is complete after the stage with lo_s = 16 J. Wave w
                // computes the extinction of layers lo_s + 2w and lo_s + 2w + 1 while the table rows
                // of the two following stages are in flight, then runs the matrix-core chunks of its
                // (row block, column group) items; the stages' layers are disjoint, so one barrier
                // per stage orders the extinction rows before their use.
                // a fixed number of stages (layers up to kPipeMaxLayers), so that the stage loop
                // unrolls into straight-line code and the memory-counter waits stay exact; stages
                // above the model's top rows (Lk = 16 ceil(L/16)) only reissue valid table loads
                constexpr int kStages = kPipeMaxLayers / kMfmaM;
                constexpr int Ltop = kPipeMaxLayers;
                const int Lk = kMfmaM * ((L + kMfmaM - 1) / kMfmaM);
                const int nJ = mfma_row_blocks(L);
                // record fields of this wave's layers (loaded above; only lanes below 2S are used)
                const int r_k = pf.k, r_kc = pf.kc;
                const T r_w = pf.w, r_rf = pf.rf;
                const T(&r_a)[kS] = pf.a;
                const double r_wc = pf.wc, r_b = pf.b;
                // this wave's items: the q-th is item q * 8 + (q odd ? 7 - wave : wave) of the
                // (J, column group) list, as in the unpipelined snake order
                int koff[4];
    #pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int it = q * kWaves + ((q & 1) ? (kWaves - 1 - wave) : wave);
                    koff[q] = (it < 4 * nJ) ? mfma_kstep_offset(L, it >> 2) : 0;
                }
                floatx4 acc[4];
    #pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
                T va0[2][kS], va1[2][kS], vb0[2][kS], vb1[2][kS];

                // table rows of stage s for this wave's two layers (padding layers reread the last
                // layer's rows, so every wave issues the same loads and the counters stay exact)
                auto issue = [&](int st, T (&v0)[2][kS], T (&v1)[2][kS]) {
    #pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int l = min(Ltop - kMfmaM * (st + 1) + 2 * wave + u, L - 1);
                        const T* p = tab + (size_t)lane_get(r_k, 2 * st + u) * t_stride + (size_t)l * l_stride;
    #pragma unroll
                        for (int i = 0; i < kS; ++i) {
                            v0[u][i] = ld_table<T, kNonTemporal>(p + i * s_stride);
                            v1[u][i] = ld_table<T, kNonTemporal>(p + i * s_stride + t_stride);
                        }
                    }
                };
                auto extinction = [&](int st, const T (&v0)[2][kS], const T (&v1)[2][kS]) {
    #pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int l = Ltop - kMfmaM * (st + 1) + 2 * wave + u;
                        if (l < L) {
                            const int i = 2 * st + u;
                            const T w = lane_get(r_w, i);
                            T e = T(0);
    #pragma unroll
                            for (int sp = 0; sp < kS; ++sp)
                                e = fma(lane_get(r_a[sp], i), fma(w, v1[u][sp] - v0[u][sp], v0[u][sp]), e);
                            if constexpr (kCia) {
                                const double* c = cia_s + lane_get(r_kc, i) * kTileNu + lane;
                                e += (T)(lane_get(r_b, i) * fma(lane_get(r_wc, i), c[kTileNu] - c[0], c[0]));
                            }
                            e = fma(lane_get(r_rf, i), sray, e);  // sray = 0 without Rayleigh
                            es[es_index<T>(l, lane)] = e;
                        }
                    }
                };
                auto chunks = [&](int st) {
                    const int lo = Ltop - kMfmaM * (st + 1);
                    float a[4][kMfmaChunk], bv[4][kMfmaChunk];
    #pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int it = q * kWaves + ((q & 1) ? (kWaves - 1 - wave) : wave);
                        const int J = it >> 2, col = it & 3;
                        if (it < 4 * nJ && kMfmaM * J <= lo && lo < Lk) {
                            const float* wa = wa_s + (size_t)(koff[q] + (lo - kMfmaM * J) / kMfmaK) * kWave + lane;
    #pragma unroll
                            for (int u = 0; u < kMfmaChunk; ++u) {
                                a[q][u] = wa[u * kWave];
                                bv[q][u] = es[es_index<T>(lo + kMfmaK * u + (lane >> 4), col * 16 + (lane & 15))];
                            }
                        }
                    }
    #pragma unroll
                    for (int u = 0; u < kMfmaChunk; ++u)
    #pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int it = q * kWaves + ((q & 1) ? (kWaves - 1 - wave) : wave);
                            if (it < 4 * nJ && kMfmaM * (it >> 2) <= lo && lo < Lk)
                                acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q][u], bv[q][u], acc[q], 0, 0, 0);
                        }
                    // row blocks completed by this stage: 1 - exp(-tau), impact-parameter weights
    #pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int it = q * kWaves + ((q & 1) ? (kWaves - 1 - wave) : wave);
                        const int J = it >> 2, col = it & 3;
                        if (it < 4 * nJ && kMfmaM * J == lo) {
                            double pp = 0.0;
    #pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                // rows past the last chord keep pp (a select, not a branch)
                                const int j = kMfmaM * J + 4 * (lane >> 4) + r;
                                const double t = pp + cw_s[min(j, L - 1)] * chord_fraction(j, jcl, acc[q][r], tau_max);
                                pp = j <= L - 2 ? t : pp;
                            }
                            pp += __shfl_xor(pp, 16);
                            pp += __shfl_xor(pp, 32);
                            if (lane < 16) part[J * kTileNu + col * 16 + (lane & 15)] = pp;
                        }
                    }
                };

                // prologue: the fragment copies (issued first), the impact-parameter weights, the
                // CIA columns, the record fields and the first two stages' table rows are all in
                // flight before the first wait. Vector-memory loads return in issue order, so once
                // a wave has waited for its stage-0 rows its fragment copies have landed too.
                issue(0, va0, va1);
                issue(1, vb0, vb1);
                // keep the stage loads ahead of the waits that the LDS stores below need
                __builtin_amdgcn_sched_barrier(0);
                flags = __builtin_amdgcn_readlane(hv, 4);
                if (m.cloud) jcl = __builtin_amdgcn_readlane(hv, 6);
                if ((int)threadIdx.x < L) cw_s[threadIdx.x] = cwv;
                if constexpr (kCia) cia_store();
                // zero rows past the last layer (read by the top stages against zero weights)
                for (int i = threadIdx.x; i < (lay.es_rows - L) * kTileNu; i += kWaves * kWave) es[L * kTileNu + i] = T(0);
                __syncthreads();
    #pragma unroll
                for (int st = 0; st < kStages; st += 2) {
                    if (st == 2 && late_round) __builtin_amdgcn_s_setprio(0);
                    extinction(st, va0, va1);
                    if (st + 2 < kStages) issue(st + 2, va0, va1);
                    __syncthreads();
                    chunks(st);
                    if (st + 1 < kStages) {
                        extinction(st + 1, vb0, vb1);
                        if (st + 3 < kStages) issue(st + 3, vb0, vb1);
                        __syncthreads();
                        chunks(st + 1);
                    }
                }
                __syncthreads();
                if (wave == 0) {
                    const double base = __hiloint2double(__builtin_amdgcn_readlane(hv, 1), __builtin_amdgcn_readlane(hv, 0));
                    const double rs2 = __hiloint2double(__builtin_amdgcn_readlane(hv, 3), __builtin_amdgcn_readlane(hv, 2));
                    double sum = base;
                    if (jcl >= L - 1) sum += cw_s[L - 1];  // the top chord lies in the deck
                    for (int J = 0; J < nJ; ++J) sum += part[J * kTileNu + lane];
                    dval = (flags & BM_FLAG_RADIUS) ? __builtin_nan("") : sum / rs2;
                }
            } else {
            // FP64: the first chord-weight chunk of this wave's first row block (block `wave`)
            // is fetched before phase 1, so that it has arrived when phase 2 starts
            using pre_t = typename std::conditional<sizeof(T) == 8, double2, float>::type;
            pre_t pre0{}, pre1{};
            if constexpr (sizeof(T) == 8) {
                if (wave * kRows <= L - 2) {
                    const double2* __restrict__ src =
                        reinterpret_cast<const double2*>(rec.wb + ((size_t)wave * L + wave * kRows) * kRows);
                    const int n_pieces = (L - wave * kRows) * kRows / 2;
                    pre0 = src[min(lane, n_pieces - 1)];
                    pre1 = src[min(lane + kWave, n_pieces - 1)];
                }
            }
            // ---- phase 1: extinction into LDS --------------------------------------------
            // wave w owns layers [w*per, (w+1)*per). Their record fields are loaded once, one
            // layer per lane, and broadcast with v_readlane, so the table loads of a group of
            // four layers are issued back to back without waiting on memory for addresses.
            const int per = (L + kWaves - 1) / kWaves;
            const int lb = wave * per;
            const int le = min(L, lb + per);
            const int mine = min(lb + lane, L - 1);
            const int r_k = rec.kidx[mine];
            const T r_w = rec.w[mine];
            const T r_rf = rec.rfac[mine];
            T r_a[kS];
    #pragma unroll
            for (int i = 0; i < kS; ++i) r_a[i] = rec.afac[i * L + mine];
            int r_kc = 0;
            double r_wc = 0.0, r_b = 0.0;
            if constexpr (kCia) {
                r_kc = rec.kcidx[mine];
                r_wc = rec.wc[mine];
                r_b = rec.bfac[mine];
            }
            for (int l0 = lb; l0 < le; l0 += 4) {
                T s0[4][kS], s1[4][kS];
                double c0[4], c1[4];
    #pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int uu = min(l0 + u, le - 1) - lb;
                    const T* p = tab + (size_t)lane_get(r_k, uu) * t_stride + (size_t)(lb + uu) * l_stride;
    #pragma unroll
                    for (int i = 0; i < kS; ++i) {
                        s0[u][i] = ld_table<T, kNonTemporal>(p + i * s_stride);
                        s1[u][i] = ld_table<T, kNonTemporal>(p + i * s_stride + t_stride);
                    }
                    if constexpr (kCia) {
                        const double* c = cia_s + lane_get(r_kc, uu) * kTileNu + lane;
                        c0[u] = c[0];
                        c1[u] = c[kTileNu];
                    }
                }
    #pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int l = l0 + u;
                    if (l < le) {
                        const int uu = l - lb;
                        const T w = lane_get(r_w, uu);
                        T e = T(0);
    #pragma unroll
                        for (int i = 0; i < kS; ++i)
                            e = fma(lane_get(r_a[i], uu), fma(w, s1[u][i] - s0[u][i], s0[u][i]), e);
                        if constexpr (kCia)
                            e += (T)(lane_get(r_b, uu) * fma(lane_get(r_wc, uu), c1[u] - c0[u], c0[u]));
                        e = fma(lane_get(r_rf, uu), sray, e);  // sray = 0 without Rayleigh
                        es[es_index<T>(l, lane)] = e;
                    }
                }
            }
            if constexpr (sizeof(T) == 4) {
                // zero rows past the last layer (read, against zero weights, by padded k-steps)
                for (int i = threadIdx.x; i < (lay.es_rows - L) * kTileNu; i += kWaves * kWave) es[L * kTileNu + i] = T(0);
            }
            if constexpr (kStageA) __builtin_amdgcn_s_waitcnt(0);  // this wave's LDS copies are done
            __syncthreads();

            // ---- phase 2: chord optical depth, 1 - exp(-tau), impact-parameter sum -------
            if constexpr (sizeof(T) == 4) {
                // items (row block J, 16-column group) in decreasing cost, dealt in snake order
                const int nJ = mfma_row_blocks(L);
                const int n_items = nJ * 4;
                for (int it = 0; it < n_items; ++it) {
                    const int round = it / kWaves, pos = it - round * kWaves;
                    const int owner = (round & 1) ? (kWaves - 1 - pos) : pos;
                    if (owner != wave) continue;
                    const int J = it >> 2, col = it & 3;
                    const int K = mfma_ksteps(L, J);  // a multiple of kMfmaChunk
                    const int brow = kMfmaM * J + (lane >> 4);
                    const int bcol = col * 16 + (lane & 15);
                    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
                    floatx4 acc2 = {0.f, 0.f, 0.f, 0.f};
                    if constexpr (kStageA) {
                        // A fragments and B from LDS
                        const float* wa = wa_s + (size_t)mfma_kstep_offset(L, J) * kWave + lane;
                        for (int ks = 0; ks < K; ks += kMfmaChunk) {
                            float ac[kMfmaChunk], bv[kMfmaChunk];
    #pragma unroll
                            for (int u = 0; u < kMfmaChunk; ++u) {
                                ac[u] = wa[(ks + u) * kWave];
                                bv[u] = es[es_index<T>(brow + kMfmaK * (ks + u), bcol)];
                            }
    #pragma unroll
                            for (int u = 0; u < kMfmaChunk; u += 2) {
                                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[u], bv[u], acc, 0, 0, 0);
                                acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[u + 1], bv[u + 1], acc2, 0, 0, 0);
                            }
                        }
                    } else {
                        // A fragments stream from L2 (coalesced, one chunk ahead), B from LDS
                        const float* ag = rec.wb + (size_t)mfma_kstep_offset(L, J) * kWave + lane;
                        float an[kMfmaChunk];
    #pragma unroll
                        for (int u = 0; u < kMfmaChunk; ++u) an[u] = ag[u * kWave];
                        for (int ks = 0; ks < K; ks += kMfmaChunk) {
                            float ac[kMfmaChunk], bv[kMfmaChunk];
    #pragma unroll
                            for (int u = 0; u < kMfmaChunk; ++u) {
                                ac[u] = an[u];
                                an[u] = ag[min(ks + kMfmaChunk + u, K - 1) * kWave];
                                bv[u] = es[es_index<T>(brow + kMfmaK * (ks + u), bcol)];
                            }
    #pragma unroll
                            for (int u = 0; u < kMfmaChunk; u += 2) {
                                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[u], bv[u], acc, 0, 0, 0);
                                acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[u + 1], bv[u + 1], acc2, 0, 0, 0);
                            }
                        }
                    }
                    acc += acc2;
                    // this lane holds rows 16J + 4(lane/16) + r of column bcol
                    double pp = 0.0;
    #pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        // rows past the last chord keep pp (a select, not a branch)
                        const int j = kMfmaM * J + 4 * (lane >> 4) + r;
                        const double t = pp + cw_s[min(j, L - 1)] * chord_fraction(j, jcl, acc[r], tau_max);
                        pp = j <= L - 2 ? t : pp;
                    }
                    pp += __shfl_xor(pp, 16);
                    pp += __shfl_xor(pp, 32);
                    if (lane < 16) part[J * kTileNu + bcol] = pp;
                }
                __syncthreads();
                if (wave == 0) {
                    double s = rec.hdr->base;
                    if (jcl >= L - 1) s += cw_s[L - 1];
                    for (int J = 0; J < nJ; ++J) s += part[J * kTileNu + lane];
                    dval = s / rec.hdr->rs2;
                }
            } else {
                // FP64: vector ALU, 8-row register blocks. The block's chord weights (layers
                // j0 .. L-1, 8 rows each, contiguous) pass through the wave's LDS chunk: two
                // coalesced 16-byte loads per lane per 32 layers, issued one chunk ahead, read
                // back as broadcasts. (Uniform scalar loads in the layer loop waited on memory
                // every few layers: the scalar-memory counter also counts the LDS reads of e,
                // so no scalar load could be kept in flight across them.)
                double acc = 0.0;
                const int nbu = (L - 1 + kRows - 1) / kRows;
                double* wst = reinterpret_cast<double*>(smem + lay.wst) + (size_t)wave * kChunkL * kRows;
                constexpr int kPieces = kChunkL * kRows / 2;  // 16-byte pieces per chunk (2 per lane)
                static_assert(kPieces == 2 * kWave, "two pieces per lane");
                for (int blk = 0; blk < nbu; ++blk) {
                    const int round = blk / kWaves, pos = blk - round * kWaves;
                    const int owner = (round & 1) ? (kWaves - 1 - pos) : pos;
                    if (owner != wave) continue;
                    const int j0 = blk * kRows;
                    T t[kRows];
    #pragma unroll
                    for (int r = 0; r < kRows; ++r) t[r] = T(0);
                    // pieces from layer j0 on; indices past the block's end are clamped to its
                    // last piece (in bounds; those layers are never read back)
                    const double2* __restrict__ src =
                        reinterpret_cast<const double2*>(rec.wb + ((size_t)blk * L + j0) * kRows);
                    const int n_pieces = (L - j0) * kRows / 2;
                    double2 nx0 = blk == wave ? pre0 : src[min(lane, n_pieces - 1)];
                    double2 nx1 = blk == wave ? pre1 : src[min(lane + kWave, n_pieces - 1)];
                    for (int c0 = j0; c0 < L; c0 += kChunkL) {
                        const double2 cur0 = nx0, cur1 = nx1;
                        if (c0 + kChunkL < L) {  // the next chunk, in flight during this one
                            const int q = (c0 + kChunkL - j0) * kRows / 2 + lane;
                            nx0 = src[min(q, n_pieces - 1)];
                            nx1 = src[min(q + kWave, n_pieces - 1)];
                        }
                        __builtin_amdgcn_wave_barrier();  // the previous chunk's reads are issued
                        reinterpret_cast<double2*>(wst)[lane] = cur0;
                        reinterpret_cast<double2*>(wst)[lane + kWave] = cur1;
                        __builtin_amdgcn_wave_barrier();
                        const int c1 = min(c0 + kChunkL, L);
                        for (int l = c0; l < c1; ++l) {
                            const T e = es[es_index<T>(l, lane)];
                            const double* w = wst + (l - c0) * kRows;
    #pragma unroll
                            for (int r = 0; r < kRows; ++r) t[r] = fma(w[r], e, t[r]);
                        }
                    }
    #pragma unroll
                    for (int r = 0; r < kRows; ++r) {
                        const int j = j0 + r;
                        if (j <= L - 2) acc += cw_s[j] * chord_fraction(j, jcl, t[r], tau_max);
                    }
                }
                part[wave * kTileNu + lane] = acc;
                __syncthreads();
                if (wave == 0) {
                    double s = rec.hdr->base;
                    if (jcl >= L - 1) s += cw_s[L - 1];
                    for (int w2 = 0; w2 < kWaves; ++w2) s += part[w2 * kTileNu + lane];
                    dval = s / rec.hdr->rs2;
                }
            }
            }  // unpipelined
        }
        if (wave == 0) {
            if (valid) dout[nu] = dval;
            dsh[lane] = dval;
        }

        // ---- phase 3: channels of this tile; chi^2 partial; last tile sums the partials ----
        if (binned == nullptr || !sg.fused_bins) return;
        __syncthreads();
        if constexpr (!kPipe) channels();
        double* bout = binned + sg.bin_off + (size_t)s_in * nbins;
        if (wave == 0) {
            double term = 0.0;
            if (own_bin) {
                double acc = 0.0;
                for (int q = 0; q < bw; ++q) acc += dsh[lane * bw + q];
                const double mean = acc / bw;
                bout[cg] = mean;
                if (want_chi2) {
                    if constexpr (!kPipe) {
                        ch_data = m.data[cg];
                        ch_err = m.err[cg];
                    }
                    const double d = (mean - ch_data) / ch_err;
                    term = d * d;
                }
            }
            if (want_chi2) {
                // fixed-order butterfly over the wave
                for (int o = 32; o > 0; o >>= 1) term += __shfl_xor(term, o);
                if (lane == 0) rec.chi2part[tile] = term;
            }
        }
    };
    if constexpr (kCompact) {
        const int n_items = *compact_count;
        for (int q = slot; q < n_items; q += slots) {
            if (q != slot) __syncthreads();  // the previous sample's LDS reads are done
            run(compact[q] - sg.first);
        }
    } else {
        run(slot);
    }
}

template <typename T, int kW, bool kNT, int kMode>
int launch_k_forward(const HostPlan& hp, const LaunchPlan& lp, size_t lds, char* ws, const int32_t* act,
                     double* depth, double* binned, double* c2, const int32_t* compact,
                     const int32_t* compact_count, int compact_slots, hipStream_t st, hipEvent_t ev0,
                     hipEvent_t ev1) {
    // a compacted launch has compact_slots sample slots per tile of its one run of samples
    // (FP32 with cached table loads)
    if (compact && (lp.n_seg != 1 || compact_slots < 1 || kNT || sizeof(T) != 4)) return BM_EINVAL;
    const dim3 grid(compact ? segment_wgs(compact_slots, lp.seg[0].tiles) : lp.total_wgs), block(kW * kWave);
    int code = BM_OK;
    // one run of samples (pipelined modes): its model moves to slot 0
    constexpr bool kHasSingle = kMode == kModePipelined;
    const bool single = kHasSingle && lp.n_seg == 1;
    LaunchPlan lp1 = lp;
    if (single) {
        lp1.model[0] = lp.model[lp.seg[0].model];
        lp1.seg[0].model = 0;
    }
    // the second dispatch round of a launch with at most two workgroups per CU (all resident
    // at once) takes a higher wave priority through its first stages
    const int n_cu = device_cu_count();
    lp1.prio_from = (n_cu > 0 && (int)grid.x <= 2 * n_cu) ? n_cu : INT_MAX;
    switch (hp.n_species) {
#define BM_FWD_GO(NS, CIA, SINGLE, COMPACT, PLAN)                                                          \
    code = ensure_dynamic_lds((const void*)k_forward<T, kW, NS, CIA, kNT, kMode, SINGLE, COMPACT>, lds);    \
    if (code != BM_OK) return code;                                                                         \
    hipExtLaunchKernelGGL((k_forward<T, kW, NS, CIA, kNT, kMode, SINGLE, COMPACT>), grid, block, lds, st, ev0, \
                          ev1, 0, PLAN, ws, act, depth, binned, c2, compact, compact_count, compact_slots);
#define BM_FWD_GO2(NS, CIA, SINGLE, PLAN)                        \
    if constexpr (!kNT && sizeof(T) == 4) {                      \
        if (compact) {                                           \
            BM_FWD_GO(NS, CIA, SINGLE, true, PLAN)               \
        } else {                                                 \
            BM_FWD_GO(NS, CIA, SINGLE, false, PLAN)              \
        }                                                        \
    } else {                                                     \
        BM_FWD_GO(NS, CIA, SINGLE, false, PLAN)                  \
    }
#define BM_FWD_LAUNCH(NS, CIA)                 \
    if constexpr (kHasSingle) {                \
        if (single) {                          \
            BM_FWD_GO2(NS, CIA, true, lp1)     \
        } else {                               \
            BM_FWD_GO2(NS, CIA, false, lp1)    \
        }                                      \
    } else {                                   \
        BM_FWD_GO2(NS, CIA, false, lp1)        \
    }
#define BM_FWD_CASE(NS)              \
    case NS:                         \
        if (hp.cia) {                \
            BM_FWD_LAUNCH(NS, true)  \
        } else {                     \
            BM_FWD_LAUNCH(NS, false) \
        }                            \
        break;
        BM_FWD_CASE(1) BM_FWD_CASE(2) BM_FWD_CASE(3) BM_FWD_CASE(4)
        BM_FWD_CASE(5) BM_FWD_CASE(6) BM_FWD_CASE(7) BM_FWD_CASE(8)
#undef BM_FWD_CASE
#undef BM_FWD_LAUNCH
#undef BM_FWD_GO2
#undef BM_FWD_GO
        default: return BM_ESHAPE;
    }
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

}  // namespace bm
