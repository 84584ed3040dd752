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
//            wavenumber, non-temporal) with no memory wait for addresses. CIA rows of
//            the tile are staged in LDS once. e[l][nu] is left in LDS.
//   phase 2  chord optical depth on the matrix cores (FP32): v_mfma_f32_16x16x4f32 over
//            16-row blocks of the triangular chord-weight matrix (A, staged in LDS) and
//            4-layer slices of e (B); items (row block, 16-column group) are dealt to
//            waves in snake order. Each finished optical depth becomes 1 - exp(-tau) and
//            is accumulated in double with its impact-parameter weight; partial sums are
//            combined in a fixed order. FP64 uses the vector ALU with 8-row blocks.
//   phase 3  the tile bins its own channels and writes its chi^2 partial; a small
//            kernel sums the partials per sample in a fixed tree.
// Workgroups are ordered XCD-aware and tile-major (see Segment) so that, in a batch,
// all samples of one tile read the same table rows from the same L2.
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

typedef float floatx4 __attribute__((ext_vector_type(4)));

// LDS layout of one forward workgroup (bytes from the start of dynamic shared memory):
//   es    extinction tile [rows][64] (FP32: L rounded up to 4 plus 16 zero rows, the
//         furthest a padded k-step reaches)
//   cw    impact-parameter weights [L] (double)
//   u     CIA rows of the tile [NTc][64] (double) during phase 1; afterwards the
//         per-row-block partial sums [blocks][64] and the tile's depths [64]
template <typename T>
struct FwdLds {
    size_t es, cw, ciat, part, bins, total;
    int es_rows;
    __host__ __device__ FwdLds(int L, int kWaves, int ntc) {
        es_rows = (sizeof(T) == 4) ? ((L + 3) & ~3) + kMfmaM : L;
        es = 0;
        size_t o = align_up(sizeof(T) * (size_t)es_rows * kTileNu, 16);
        cw = o;
        o = align_up(o + sizeof(double) * (size_t)L, 16);
        ciat = o;
        part = o;
        const int nparts = (sizeof(T) == 4) ? mfma_row_blocks(L) : kWaves;
        bins = part + sizeof(double) * (size_t)nparts * kTileNu;
        size_t u1 = sizeof(double) * (size_t)ntc * kTileNu;
        size_t u2 = bins + sizeof(double) * kTileNu - o;
        o += (u1 > u2 ? u1 : u2);
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

template <typename T, int kWaves, int kS, bool kCia, bool kNonTemporal>
__global__ void __launch_bounds__(kWaves * kWave)
    k_forward(LaunchPlan plan, char* __restrict__ ws, const int32_t* __restrict__ active,
              double* __restrict__ depth, double* __restrict__ binned, double* __restrict__ chi2) {
    extern __shared__ __align__(16) char smem[];
    const int si = plan.segment_of_wg(blockIdx.x);
    const Segment& sg = plan.seg[si];
    const ModelDev& m = plan.model[sg.model];
    // XCD-aware order: workgroup g runs on XCD g % 8; each XCD sweeps its own contiguous
    // tile range and runs all samples of a tile back to back (shared table rows in L2)
    const int g = blockIdx.x - sg.tile_begin;
    const int kx = g / kXcds;
    const int tile = (g % kXcds) * sg.tiles_per_xcd + kx / sg.count;
    const int s_in = kx % sg.count;
    if (tile >= sg.tiles) return;  // padding workgroup of the XCD split
    const int b = sg.first + s_in;
    if (active && !active[b]) return;  // sample not requested in this call
    const int L = m.L, Nnu = m.Nnu;
    const RecordView<T> rec(ws + sg.ws_off + (size_t)s_in * sg.rec_bytes, kS, L);
    const FwdLds<T> lay(L, kWaves, plan.max_ntc);

    const int lane = threadIdx.x & (kWave - 1);
    // the wave index is uniform across a wave; readfirstlane lets the compiler keep the
    // layer loops and every per-layer record load on the scalar unit
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int nu = tile * sg.tile_w + lane;
    const bool valid = lane < sg.tile_w && nu < Nnu;
    const int nu_c = valid ? nu : min(tile * sg.tile_w, Nnu - 1);

    T* es = reinterpret_cast<T*>(smem + lay.es);
    double* part = reinterpret_cast<double*>(smem + lay.part);
    double* dsh = reinterpret_cast<double*>(smem + lay.bins);
    double* dout = depth + sg.depth_off + (size_t)s_in * Nnu;
    const int flags = rec.hdr->flags;
    double dval = __builtin_nan("");  // this lane's depth (wave 0)

    if (!(flags & BM_FLAG_RADIUS)) {
        // impact-parameter weights to LDS (read per optical depth in phase 2)
        double* cw_s = reinterpret_cast<double*>(smem + lay.cw);
        for (int i = threadIdx.x; i < L; i += kWaves * kWave) cw_s[i] = rec.cw[i];
        // this tile's columns of every CIA temperature row (read by many layers); the
        // loads are all issued before the first store
        double* cia_s = reinterpret_cast<double*>(smem + lay.ciat);
        if constexpr (kCia) {
            constexpr int kMaxPer = BM_MAX_TEMPS * kTileNu / (kWaves * kWave);
            const int n = m.NTc * kTileNu;
            double cv[kMaxPer];
#pragma unroll
            for (int q = 0; q < kMaxPer; ++q) {
                const int i = min((int)threadIdx.x + q * kWaves * kWave, n - 1);
                const int col = min(tile * sg.tile_w + (i % kTileNu), Nnu - 1);
                cv[q] = m.cia[(size_t)(i / kTileNu) * Nnu + col];
            }
#pragma unroll
            for (int q = 0; q < kMaxPer; ++q) {
                const int i = threadIdx.x + q * kWaves * kWave;
                if (i < n) cia_s[i] = cv[q];
            }
        }
        __syncthreads();

        // ---- phase 1: extinction into LDS --------------------------------------------
        // wave w owns layers [w*per, (w+1)*per). Their record fields are loaded once, one
        // layer per lane, and broadcast with v_readlane, so the table loads of a group of
        // four layers are issued back to back without waiting on memory for addresses.
        const T* __restrict__ sig = static_cast<const T*>(m.sigma);
        const size_t t_stride = (size_t)L * Nnu;
        const size_t s_stride = (size_t)m.NT * t_stride;
        const int per = (L + kWaves - 1) / kWaves;
        const int lb = wave * per;
        const int le = min(L, lb + per);
        const int mine = min(lb + lane, L - 1);
        const int r_k = rec.kidx[mine];
        const T r_w = rec.w[mine];
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
                const T* p = sig + (size_t)lane_get(r_k, uu) * t_stride + (size_t)(lb + uu) * Nnu + nu_c;
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
                    es[es_index<T>(l, lane)] = e;
                }
            }
        }
        if constexpr (sizeof(T) == 4) {
            // zero rows past the last layer (read, against zero weights, by padded k-steps)
            for (int i = threadIdx.x; i < (lay.es_rows - L) * kTileNu; i += kWaves * kWave) es[L * kTileNu + i] = T(0);
        }
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
                // A fragments stream from L2 (coalesced, one chunk ahead), B from LDS. (Staging
                // them in LDS measured slower: it holds registers through phase 1.)
                const float* ag = rec.wb + (size_t)mfma_kstep_offset(L, J) * kWave + lane;
                const int brow = kMfmaM * J + (lane >> 4);
                const int bcol = col * 16 + (lane & 15);
                floatx4 acc = {0.f, 0.f, 0.f, 0.f};
                floatx4 acc2 = {0.f, 0.f, 0.f, 0.f};
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
                acc += acc2;
                // this lane holds rows 16J + 4(lane/16) + r of column bcol
                double pp = 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = kMfmaM * J + 4 * (lane >> 4) + r;
                    if (j <= L - 2) pp += cw_s[j] * (double)(-expm1f(-acc[r]));
                }
                pp += __shfl_xor(pp, 16);
                pp += __shfl_xor(pp, 32);
                if (lane < 16) part[J * kTileNu + bcol] = pp;
            }
            __syncthreads();
            if (wave == 0) {
                double s = rec.hdr->base;
                for (int J = 0; J < nJ; ++J) s += part[J * kTileNu + lane];
                dval = s / rec.hdr->rs2;
            }
        } else {
            // FP64: vector ALU, 8-row register blocks, chord weights as uniform loads
            double acc = 0.0;
            const int nbu = (L - 1 + kRows - 1) / kRows;
            for (int blk = 0; blk < nbu; ++blk) {
                const int round = blk / kWaves, pos = blk - round * kWaves;
                const int owner = (round & 1) ? (kWaves - 1 - pos) : pos;
                if (owner != wave) continue;
                const int j0 = blk * kRows;
                T t[kRows];
#pragma unroll
                for (int r = 0; r < kRows; ++r) t[r] = T(0);
                const T* __restrict__ wcol = rec.wb + (size_t)blk * L * kRows;
                for (int l = j0; l < L; ++l) {
                    const T e = es[es_index<T>(l, lane)];
#pragma unroll
                    for (int r = 0; r < kRows; ++r) t[r] = fma(wcol[l * kRows + r], e, t[r]);
                }
#pragma unroll
                for (int r = 0; r < kRows; ++r) {
                    const int j = j0 + r;
                    if (j <= L - 2) acc += cw_s[j] * (double)(-dev_expm1(-t[r]));
                }
            }
            part[wave * kTileNu + lane] = acc;
            __syncthreads();
            if (wave == 0) {
                double s = rec.hdr->base;
                for (int w2 = 0; w2 < kWaves; ++w2) s += part[w2 * kTileNu + lane];
                dval = s / rec.hdr->rs2;
            }
        }
    }
    if (wave == 0) {
        if (valid) dout[nu] = dval;
        dsh[lane] = dval;
    }

    // ---- phase 3: channels of this tile; chi^2 partial; last tile sums the partials ----
    if (binned == nullptr || !sg.fused_bins) return;
    __syncthreads();
    const int bw = m.bin_width;
    const int nbt = sg.tile_w / bw;   // whole channels per tile
    const int nbins = Nnu / bw;
    const bool want_chi2 = (chi2 != nullptr) && m.data && m.err;
    double* bout = binned + sg.bin_off + (size_t)s_in * nbins;
    if (wave == 0) {
        double term = 0.0;
        const int cg = tile * nbt + lane;
        if (lane < nbt && cg < nbins) {
            double acc = 0.0;
            for (int q = 0; q < bw; ++q) acc += dsh[lane * bw + q];
            const double mean = acc / bw;
            bout[cg] = mean;
            if (want_chi2) {
                const double d = (mean - m.data[cg]) / m.err[cg];
                term = d * d;
            }
        }
        if (want_chi2) {
            // fixed-order butterfly over the wave
            for (int o = 32; o > 0; o >>= 1) term += __shfl_xor(term, o);
            if (lane == 0) rec.chi2part[tile] = term;
        }
    }
}

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

static size_t record_bytes(const bm_model& m, int tiles) {
    return m.dtype == BM_F32 ? record_bytes_t<float>(m.n_species, m.n_layers, tiles)
                             : record_bytes_t<double>(m.n_species, m.n_layers, tiles);
}

// Split a batch into launch plans of at most kMaxSegments same-model runs.
struct HostPlan {
    std::vector<LaunchPlan> plans;
    std::vector<int> first_sample;   // first sample of each plan
    std::vector<int> n_samples;      // samples of each plan
    size_t ws_bytes = 0;
    int max_L = 0;
    int n_species = 0;
    bool cia = false;
    int max_ntc = 0;          // largest CIA temperature grid (LDS staging rows)
    int total_samples = 0;
    size_t max_entries = 0;   // chord-weight entries of the largest record
};

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
    }
    hp.n_species = models[0].n_species;
    hp.cia = models[0].n_temp_cia > 0;
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
            s.fused_bins = (md.bin_width > 0 && md.bin_width <= kTileNu) ? 1 : 0;
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
    hp.ws_bytes = ws;
    hp.total_samples = B;
    return BM_OK;
}

constexpr int kFwdWaves = 8;

template <typename T>
static size_t forward_lds_bytes(int max_L, int max_ntc) {
    return FwdLds<T>(max_L, kFwdWaves, max_ntc).total;
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

// Raise a kernel's dynamic-LDS ceiling once per device (hipFuncSetAttribute is host work
// that the per-call path should not repeat).
static int ensure_dynamic_lds(const void* fn, size_t bytes) {
    if (bytes <= 48 * 1024) return BM_OK;
    struct Entry { const void* fn; int dev; size_t bytes; };
    static Entry cache[64];
    static int n_cache = 0;
    int dev = 0;
    BM_CHECK_HIP(hipGetDevice(&dev));
    for (int i = 0; i < n_cache; ++i)
        if (cache[i].fn == fn && cache[i].dev == dev && cache[i].bytes >= bytes) return BM_OK;
    BM_CHECK_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    if (n_cache < 64) cache[n_cache++] = Entry{fn, dev, bytes};
    return BM_OK;
}

template <typename T>
static int launch_forward(const HostPlan& hp, const double* params, int stride, const int32_t* active,
                          double* depth, double* binned, double* chi2, int32_t* flags, char* ws, hipStream_t st) {
    const size_t lds = forward_lds_bytes<T>(hp.max_L, hp.max_ntc);
    if (lds > device_lds_limit()) return BM_ESHAPE;
    int st_code = BM_OK;
    for (size_t p = 0; p < hp.plans.size(); ++p) {
        const LaunchPlan& lp = hp.plans[p];
        const int b0 = hp.first_sample[p];
        const int nb = hp.n_samples[p];
        // Segment offsets inside a plan are absolute (workspace, depth, binned); sample
        // indices are relative to the plan, so params/flags/chi2 are shifted here.
        const int32_t* act = active ? active + b0 : nullptr;
        hipLaunchKernelGGL((k_atm_prep<T>), dim3(nb, prep_slices(hp, nb)), dim3(kAtmThreads), 0, st, lp,
                           params + (size_t)b0 * stride, stride, act, ws, flags + b0);
        BM_CHECK_HIP(hipGetLastError());
        double* c2 = chi2 ? chi2 + b0 : nullptr;
        const dim3 grid(lp.total_wgs), block(kFwdWaves * kWave);
        switch (hp.n_species) {
#define BM_FWD_LAUNCH(NS, CIA)                                                                         \
    st_code = ensure_dynamic_lds((const void*)k_forward<T, kFwdWaves, NS, CIA, true>, lds);             \
    if (st_code != BM_OK) return st_code;                                                              \
    hipLaunchKernelGGL((k_forward<T, kFwdWaves, NS, CIA, true>), grid, block, lds, st, lp, ws, act, depth, binned, c2);
#define BM_FWD_CASE(NS)                  \
    case NS:                             \
        if (hp.cia) {                    \
            BM_FWD_LAUNCH(NS, true)      \
        } else {                         \
            BM_FWD_LAUNCH(NS, false)     \
        }                                \
        break;
            BM_FWD_CASE(1) BM_FWD_CASE(2) BM_FWD_CASE(3) BM_FWD_CASE(4)
            BM_FWD_CASE(5) BM_FWD_CASE(6) BM_FWD_CASE(7) BM_FWD_CASE(8)
#undef BM_FWD_CASE
#undef BM_FWD_LAUNCH
            default: return BM_ESHAPE;
        }
        BM_CHECK_HIP(hipGetLastError());
        if (c2 && binned) {
            bool any_fused = false;
            for (int si = 0; si < lp.n_seg; ++si) any_fused |= lp.seg[si].fused_bins != 0;
            if (any_fused) {
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
                                const double* params, int param_stride, int B, const int32_t* active,
                                double* depth, double* binned, double* chi2, int32_t* flags, void* workspace,
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
        return launch_forward<float>(hp, params, param_stride, active, depth, binned, chi2, flags, (char*)workspace, s);
    return launch_forward<double>(hp, params, param_stride, active, depth, binned, chi2, flags, (char*)workspace, s);
}
