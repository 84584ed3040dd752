// Steps a1-a2 of the forward model on the GPU: parameters -> per-layer temperature,
// composition, number densities and hydrostatic radii (Sec. 3 profile generator;
// Sec. 6.2 radius at the reference pressure; Sec. 6.3 / Sec. 7 parameterisation),
// plus the per-sample record consumed by the fused forward kernel: T-interpolation
// brackets, density factors, FP64 chord weights rounded once to the compute type
// (laid out as matrix-core A fragments in FP32), and the impact-parameter weights.
#include "bm_forward.h"

namespace bm {

// One workgroup evaluates one sample; layer l is owned by thread l (L <= BM_MAX_LAYERS).
// The work is a chain of short dependent steps, so it is laid out for latency: every
// memory load is issued before the first value is used, the sample's constants (which
// depend only on its parameters) are evaluated redundantly by every thread in registers
// instead of by one thread behind a barrier, and interpolation brackets are fixed-length
// binary searches.
struct AtmShared {
    double tgrid[kWave];      // temperature grids (BM_MAX_TEMPS <= 64 points)
    double tgrid_cia[kWave];
    double temp[BM_MAX_LAYERS];
    double radius[BM_MAX_LAYERS];
    double ndens[BM_MAX_LAYERS];
    double lnp[BM_MAX_LAYERS];
    double scan[BM_MAX_LAYERS];
    double wave_tot[kAtmThreads / kWave];
    double iref;
    int flags;
    int jcloud;  // largest layer at or below the cloud top (-1: none or no cloud deck)
};

static_assert(BM_MAX_TEMPS <= kWave, "temperature grids are loaded one point per lane");

// the sample's constants, held by every thread
struct AtmSample {
    double x[BM_MAX_SPECIES];  // absorber mixing ratios (the first S)
    double x_h2;
    double mu;                 // mean molecular mass, amu
};

// No per-layer work for the record's helpers (k_atmosphere).
struct NoSideWork {
    __device__ void operator()(int, int) const {}
};

// Threads with no layer of their own once the temperatures are known: with 2 L <= 256,
// threads 128 + l; they run side(phase, l) for phases 0, 1, 2 inside the three barrier
// intervals of the radius computation, while the lower threads scan and solve for radii.
__device__ inline bool atm_has_helpers(int L) { return 2 * L <= kAtmThreads; }

// tg, tgc: this lane's points of the opacity and CIA temperature grids (loaded by the
// caller), stored to shared memory before the first barrier; storing them here keeps
// their loads issued with the atmosphere's own instead of sunk into their later use
template <typename Side = NoSideWork>
__device__ void atm_compute(const ModelDev& m, const double* __restrict__ theta_g, AtmShared& sh, AtmSample& a,
                            double tg = 0.0, double tgc = 0.0, Side side = Side()) {
    const int tid = threadIdx.x;
    const int L = m.L, S = m.S;
    const int ntp = (m.tp_mode == BM_TP_ISOTHERMAL) ? 1 : 5;
    const int np = ntp + S + 1 + m.cloud;
    // with L <= 128 the Line-2013 profile's two xi() terms of layer l are evaluated by
    // threads l and l + 128 (a dependent chain half as long)
    const bool split = (m.tp_mode == BM_TP_LINE2013) && (2 * L <= kAtmThreads);
    const int lay = split ? (tid & (kAtmThreads / 2 - 1)) : tid;
    const bool upper = split && tid >= kAtmThreads / 2;
    // every load first: this thread's layer pressure and the sample's parameters (the
    // same addresses for the whole workgroup; indices clamped, so all are issued at once)
    const double p = m.p_bar[min(lay, L - 1)];
    double th[5], xt[BM_MAX_SPECIES];
#pragma unroll
    for (int i = 0; i < 5; ++i) th[i] = theta_g[min(i, np - 1)];
#pragma unroll
    for (int i = 0; i < BM_MAX_SPECIES; ++i) xt[i] = theta_g[min(ntp + i, np - 1)];
    const double r_param = theta_g[ntp + S];
    const double cloud_param = theta_g[np - 1];
    const double lnref = log(m.pl.p_ref_bar);
    // per-sample constants
    int flags = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i)
        if (i < ntp && !isfinite(th[i])) flags |= BM_FLAG_NONFINITE;
#pragma unroll
    for (int i = 0; i < BM_MAX_SPECIES; ++i)
        if (i < S && !isfinite(xt[i])) flags |= BM_FLAG_NONFINITE;
    if (!isfinite(r_param) || (m.cloud && !isfinite(cloud_param))) flags |= BM_FLAG_NONFINITE;
    double total = 0.0;
#pragma unroll
    for (int i = 0; i < BM_MAX_SPECIES; ++i) {
        a.x[i] = (i < S) ? pow10_(xt[i]) : 0.0;
        if (i < S) total += a.x[i];
    }
    if (total >= 1.0) flags |= BM_FLAG_SUM_X;
    double fill = 1.0 - total;
    if (fill < 0.0) fill = 0.0;
    a.x_h2 = m.pl.h2_frac * fill;
    const double x_he = (1.0 - m.pl.h2_frac) * fill;
    double mu = 0.0;
#pragma unroll
    for (int i = 0; i < BM_MAX_SPECIES; ++i)
        if (i < S) mu += a.x[i] * m.mass[i];
    mu += a.x_h2 * m.pl.m_h2_amu + x_he * m.pl.m_he_amu;
    a.mu = mu;
    Line2013Consts tp{};
    if (m.tp_mode == BM_TP_LINE2013) tp = line2013_consts(th, m.pl);
    if (tid == 0) {
        sh.flags = flags;
        sh.jcloud = -1;
    }
    // every wave writes the same grid values (no branch for the loads to sink into)
    sh.tgrid[tid & (kWave - 1)] = tg;
    sh.tgrid_cia[tid & (kWave - 1)] = tgc;
    // temperature, number density and ln p per layer
    if (split) {
        const double tau = line2013_tau(p, tp);
        double xi = 0.0;
        if (lay < L) xi = line2013_xi(upper ? tp.g2 : tp.g1, tau);
        if (upper && lay < L) sh.scan[lay] = xi;  // scratch until the radius scan
        if (!upper && lay < L) sh.lnp[lay] = log(p);
        __syncthreads();
        if (tid < L) {
            const double t = line2013_temperature_xi(tau, xi, sh.scan[tid], tp);
            sh.temp[tid] = t;
            sh.ndens[tid] = p * kBar / (kBoltz * t);
        }
    } else if (tid < L) {
        const double t = (m.tp_mode == BM_TP_ISOTHERMAL) ? th[0] : line2013_temperature_c(p, tp);
        sh.temp[tid] = t;
        sh.ndens[tid] = p * kBar / (kBoltz * t);
        sh.lnp[tid] = log(p);
    }
    __syncthreads();
    if (tid < L && !(isfinite(sh.temp[tid]) && sh.temp[tid] > 0.0)) atomicOr(&sh.flags, BM_FLAG_NONFINITE);
    // gray cloud deck: the largest layer with p_l >= p_cloud (any layer order)
    if (m.cloud && tid < L && p >= pow10_(cloud_param)) atomicMax(&sh.jcloud, tid);
    const bool helper = atm_has_helpers(L) && tid >= kAtmThreads / 2;
    const int hl = tid - kAtmThreads / 2;
    // hydrostatic radii: 1/r_l = 1/R_ref + k_B/(GM mu m_u) (I_l - I_ref), with I the
    // exact integral of the piecewise-linear (in ln p) temperature from layer 0:
    // segment integrals, an inclusive scan within each wave (shuffles), then each wave
    // adds the totals of the waves before it (helper waves hold no layers)
    {
        double v = (tid > 0 && tid < L) ? (sh.lnp[tid] - sh.lnp[tid - 1]) * 0.5 * (sh.temp[tid - 1] + sh.temp[tid]) : 0.0;
        const int lane = tid & (kWave - 1), w = tid / kWave;
        if (helper) {
            if (hl < L) side(0, hl);
        } else {
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const double u = __shfl_up(v, off, kWave);
                if (lane >= off) v += u;
            }
            if (lane == kWave - 1) sh.wave_tot[w] = v;
        }
        __syncthreads();
        if (helper) {
            if (hl < L) side(1, hl);
        } else {
            for (int q = 0; q < w; ++q) v += sh.wave_tot[q];
            if (tid < L) sh.scan[tid] = v;
        }
    }
    __syncthreads();
    // the layer m with ln p_m >= ln p_ref > ln p_{m+1} (pressures decrease with l; m is
    // clamped to [0, L-2], i.e. linear extrapolation outside the grid)
    if (tid < L - 1) {
        // exactly one thread owns m: the layers with ln p >= ln p_ref form a prefix
        const bool owner = (tid == 0 || sh.lnp[tid] >= lnref) && (tid == L - 2 || sh.lnp[tid + 1] < lnref);
        if (owner) {
            const int mref = tid;
            const double la = sh.lnp[mref], lb = sh.lnp[mref + 1];
            const double tref = sh.temp[mref] + (sh.temp[mref + 1] - sh.temp[mref]) * (lnref - la) / (lb - la);
            sh.iref = sh.scan[mref] + (lnref - la) * 0.5 * (sh.temp[mref] + tref);
        }
    }
    if (helper && hl < L) side(2, hl);
    __syncthreads();
    if (tid < L) {
        const double gm = m.pl.g_nom * m.pl.r_nom_cm * m.pl.r_nom_cm;
        const double coef = kBoltz / (gm * a.mu * kAmu);
        const double rref = r_param * kRJup;
        const double inv_r = 1.0 / rref + coef * (sh.scan[tid] - sh.iref);
        if (!(inv_r > 0.0)) {
            atomicOr(&sh.flags, BM_FLAG_RADIUS);
            sh.radius[tid] = NAN;
        } else {
            sh.radius[tid] = 1.0 / inv_r;
        }
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kAtmThreads)
    k_atmosphere(ModelDev m, const double* __restrict__ params, int stride, double* temp, double* n_species,
                 double* n_h2, double* radius, int32_t* flags) {
    __shared__ AtmShared sh;
    AtmSample a;
    const int b = blockIdx.x;
    atm_compute(m, params + (size_t)b * stride, sh, a);
    const int tid = threadIdx.x;
    const int L = m.L;
    if (tid < L) {
        temp[(size_t)b * L + tid] = sh.temp[tid];
        radius[(size_t)b * L + tid] = sh.radius[tid];
        n_h2[(size_t)b * L + tid] = a.x_h2 * sh.ndens[tid];
#pragma unroll
        for (int i = 0; i < BM_MAX_SPECIES; ++i)
            if (i < m.S) n_species[((size_t)b * m.S + i) * L + tid] = a.x[i] * sh.ndens[tid];
    }
    if (tid == 0) flags[b] = sh.flags;
}

// Interpolation bracket of t on a strictly increasing grid of n <= 64 points in shared
// memory: k = the largest index with grid[k] <= t, clamped to [0, n-2] (0 when none, or
// for a NaN t); w = (t - grid[k]) / (grid[k+1] - grid[k]) clamped to [0, 1] (0 for a NaN
// t). Returns true when t lies outside [grid[0], grid[n-1]]. A binary search with a fixed
// six steps (2^6 >= n - 1), so that the dependent chain is six shared-memory reads.
__device__ inline bool bracket_search(const double* grid, int n, double t, int* k_out, double* w_out) {
    int lo = 0, hi = n - 2;  // the answer lies in [lo, hi]
#pragma unroll
    for (int step = 0; step < 6; ++step) {
        const int mid = (lo + hi + 1) >> 1;  // in (lo, hi] while lo < hi
        const bool le = grid[mid] <= t;
        if (lo < hi) {
            lo = le ? mid : lo;
            hi = le ? hi : mid - 1;
        }
    }
    const double g0 = grid[lo], g1 = grid[lo + 1];
    double w = (t - g0) / (g1 - g0);
    const bool clamped = !(grid[0] <= t && t <= grid[n - 1]);
    w = w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
    if (!(w == w)) w = 0.0;  // NaN temperature: flagged elsewhere
    *k_out = lo;
    *w_out = w;
    return clamped;
}

// Chord weight of row j (impact parameter r_j) on layer l, from the trapezoid in path
// length: W[j][l] = [l <= L-2](s_{j,l+1} - s_{j,l}) + [l >= j+1](s_{j,l} - s_{j,l-1}),
// s_{j,l} = sqrt(r_l^2 - r_j^2) (zero for l = j), and W = 0 outside j <= L-2, j <= l < L.
// Double precision.
__device__ inline double chord_weight(const double* r, int L, int j, int l) {
    if (j > L - 2 || l < j || l >= L) return 0.0;
    const double s_l = (l == j) ? 0.0 : half_chord(r[l], r[j]);
    double w = 0.0;
    if (l <= L - 2) w += half_chord(r[l + 1], r[j]) - s_l;
    if (l >= j + 1) w += s_l - ((l - 1 == j) ? 0.0 : half_chord(r[l - 1], r[j]));
    return w;
}

// Per-sample record for the fused forward kernel. Grid: B samples x P slices. Every
// workgroup of a sample evaluates its atmosphere (a latency-bound chain of a few us);
// slice p fills 1/P of the chord weights, slice 0 also the per-layer fields.
// A masked call with a device-built list of its requested samples (compact, its count at
// *compact_count) launches a few sample slots instead of every sample: slot x takes list
// entries x, x + gridDim.x, ... in turn.
template <typename T, bool kSingle, bool kMasked>
__global__ void __launch_bounds__(kAtmThreads)
    k_atm_prep(LaunchPlan plan, const double* __restrict__ params, int stride, const int32_t* __restrict__ active,
               char* __restrict__ ws, int32_t* __restrict__ flags_out, int32_t* __restrict__ compact,
               const int32_t* __restrict__ compact_count, int build_n) {
    __shared__ AtmShared sh;
  auto one = [&](const int b) {
    const int slice = blockIdx.y, n_slices = gridDim.y;
    // a single-segment plan keeps its model in slot 0, so the model's fields sit at fixed
    // kernel-argument offsets and are fetched in one round
    const int si = kSingle ? 0 : plan.segment_of_sample(b);
    const Segment& sg = plan.seg[si];
    const ModelDev& m = plan.model[kSingle ? 0 : sg.model];
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    // the temperature grids, one point per lane, in flight with the atmosphere's own
    // loads (without CIA the second load rereads the first grid)
    const bool cia = m.NTc > 0;
    const double tg = m.temp[min(lane, m.NT - 1)];
    const double tgc = (cia ? m.temp_cia : m.temp)[min(lane, (cia ? m.NTc : m.NT) - 1)];
    const int L = m.L;
    RecordView<T> rec(ws + sg.ws_off + (size_t)(b - sg.first) * sg.rec_bytes, m.S, L);
    // slice 0 writes the per-layer record fields: interpolation brackets (temperature and
    // CIA grids), then density factors, by the helper threads while the radii are solved
    // (or by the layer's own thread afterwards when there are no helpers)
    AtmSample a;
    int k = 0, kc = 0, fl = 0;
    double w = 0.0, wc = 0.0;
    auto fields = [&](int phase, int l) {
        if (slice != 0) return;
        if (phase == 0) {
            // both searches back to back, with no branch between them, so that their
            // dependent read chains overlap (without CIA the second repeats the first)
            const double t = sh.temp[l];
            const bool c1 = bracket_search(sh.tgrid, m.NT, t, &k, &w);
            int kc2;
            double wc2;
            const bool c2 = bracket_search(cia ? sh.tgrid_cia : sh.tgrid, cia ? m.NTc : m.NT, t, &kc2, &wc2);
            if (c1 || (cia && c2)) fl |= BM_FLAG_T_CLAMP;
            if (cia) {
                kc = kc2;
                wc = wc2;
            }
        } else if (phase == 1) {
            rec.kidx[l] = k;
            rec.kcidx[l] = kc;
            rec.w[l] = (T)w;
            rec.wc[l] = wc;
            const double nh2 = a.x_h2 * sh.ndens[l];
            rec.bfac[l] = nh2 * nh2;
            rec.rfac[l] = (T)nh2;
            rec.tl[l] = sh.temp[l];
        } else {
#pragma unroll
            for (int i = 0; i < BM_MAX_SPECIES; ++i)
                if (i < m.S) rec.afac[i * L + l] = (T)(a.x[i] * sh.ndens[l]);
            if (fl) atomicOr(&sh.flags, fl);
        }
    };
    atm_compute(m, params + (size_t)b * stride, sh, a, tg, tgc, fields);
    const double* r = sh.radius;

    if (slice == 0) {
        if (tid < L) {
            if (!atm_has_helpers(L))
                for (int phase = 0; phase < 3; ++phase) fields(phase, tid);
            // impact-parameter quadrature weight of f_j (trapezoid in b)
            double c;
            if (tid == 0)
                c = (r[1] - r[0]) * r[0];
            else if (tid == L - 1)
                c = (r[L - 1] - r[L - 2]) * r[L - 1];
            else
                c = r[tid] * (r[tid + 1] - r[tid - 1]);
            rec.cw[tid] = c;
            rec.rl[tid] = r[tid];
        }
        __syncthreads();
        if (tid == 0) {
            rec.hdr->base = r[0] * r[0];
            rec.hdr->rs2 = m.pl.rs_cm * m.pl.rs_cm;
            rec.hdr->flags = sh.flags;
            rec.hdr->jcloud = sh.jcloud;
            flags_out[b] = sh.flags;
        }
    }
    const int n = (int)chord_weight_entries<T>(L);
    const int per = (n + n_slices - 1) / n_slices;
    const int i0 = slice * per, i1 = min(n, i0 + per);
    for (int idx = i0 + tid; idx < i1; idx += kAtmThreads) {
        int j, l;
        if constexpr (sizeof(T) == 4) {
            // A fragments of v_mfma_f32_16x16x4f32: entry (kstep, lane) of row block J
            // holds W[16J + lane % 16][16J + 4 kstep + lane / 16]
            const int kg = idx / kWave, lane = idx % kWave;
            int J = 0;
            while (mfma_kstep_offset(L, J + 1) <= kg) ++J;
            const int off = mfma_kstep_offset(L, J);
            j = kMfmaM * J + (lane % kMfmaM);
            l = kMfmaM * J + kMfmaK * (kg - off) + lane / kMfmaM;
        } else {
            // 8-row blocks [nb][L][8] for the vector-ALU path
            const int rr = idx % kRows;
            l = (idx / kRows) % L;
            j = (idx / (kRows * L)) * kRows + rr;
        }
        rec.wb[idx] = (T)chord_weight(r, L, j, l);
    }
  };
    if constexpr (kMasked) {
        if (compact && build_n > 0) {
            // the list of requested samples (ascending), built by every workgroup from the
            // B flags; the first workgroup also writes it, with its length after the B
            // entries, for the fused kernel
            __shared__ int32_t lst[kPrepListMax];
            __shared__ int tsum[kAtmThreads / kWave];
            constexpr int kPer = kPrepListMax / kAtmThreads;
            int mine[kPer], c = 0;
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                const int b = threadIdx.x * kPer + j;
                mine[j] = (b < build_n && active[b] != 0) ? b : -1;
                c += mine[j] >= 0;
            }
            // exclusive prefix of the counts over the threads: a scan within each wave, then
            // the totals of the waves before
            const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
            int incl = c;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const int v = __shfl_up(incl, o, kWave);
                if (lane >= o) incl += v;
            }
            if (lane == kWave - 1) tsum[w] = incl;
            __syncthreads();
            int off = incl - c;
            for (int q = 0; q < w; ++q) off += tsum[q];
#pragma unroll
            for (int j = 0; j < kPer; ++j)
                if (mine[j] >= 0) lst[off++] = mine[j];
            int n_items = 0;
            for (int q = 0; q < kAtmThreads / kWave; ++q) n_items += tsum[q];
            __syncthreads();
            if (blockIdx.x == 0 && blockIdx.y == 0) {
                for (int q = threadIdx.x; q < n_items; q += kAtmThreads) compact[q] = lst[q];
                if (threadIdx.x == 0) compact[build_n] = n_items;
            }
            for (int q = blockIdx.x; q < n_items; q += gridDim.x) {
                if (q != (int)blockIdx.x) __syncthreads();  // the previous sample's shared reads are done
                one(lst[q]);
            }
            return;
        }
        if (compact) {
            const int n_items = *compact_count;
            for (int q = blockIdx.x; q < n_items; q += gridDim.x) {
                if (q != (int)blockIdx.x) __syncthreads();  // the previous sample's shared reads are done
                one(compact[q]);
            }
            return;
        }
        if (!active[blockIdx.x]) return;  // sample not requested in this call
    }
    one(blockIdx.x);
}

template __global__ void k_atm_prep<float, true, true>(LaunchPlan, const double*, int, const int32_t*, char*, int32_t*,
                                                      int32_t*, const int32_t*, int);
template __global__ void k_atm_prep<float, true, false>(LaunchPlan, const double*, int, const int32_t*, char*, int32_t*,
                                                      int32_t*, const int32_t*, int);
template __global__ void k_atm_prep<float, false, true>(LaunchPlan, const double*, int, const int32_t*, char*, int32_t*,
                                                      int32_t*, const int32_t*, int);
template __global__ void k_atm_prep<float, false, false>(LaunchPlan, const double*, int, const int32_t*, char*, int32_t*,
                                                      int32_t*, const int32_t*, int);
template __global__ void k_atm_prep<double, true, true>(LaunchPlan, const double*, int, const int32_t*, char*, int32_t*,
                                                      int32_t*, const int32_t*, int);
template __global__ void k_atm_prep<double, true, false>(LaunchPlan, const double*, int, const int32_t*, char*, int32_t*,
                                                      int32_t*, const int32_t*, int);
template __global__ void k_atm_prep<double, false, true>(LaunchPlan, const double*, int, const int32_t*, char*, int32_t*,
                                                      int32_t*, const int32_t*, int);
template __global__ void k_atm_prep<double, false, false>(LaunchPlan, const double*, int, const int32_t*, char*, int32_t*,
                                                      int32_t*, const int32_t*, int);

}  // namespace bm

extern "C" int bm_atmosphere(const bm_model* model, const double* params, int param_stride, int B,
                             double* temp, double* n_species, double* n_h2, double* radius,
                             int32_t* flags, void* stream) {
    using namespace bm;
    if (!model || !params || !temp || !n_species || !n_h2 || !radius || !flags) return BM_EINVAL;
    int st = validate_model(*model, /*need_tables=*/false);
    if (st != BM_OK) return st;
    if (B < 0 || param_stride < bm_n_params(model)) return BM_ESHAPE;
    if (B == 0) return BM_OK;
    ModelDev m = to_device_view(*model);
    hipLaunchKernelGGL(k_atmosphere, dim3(B), dim3(kAtmThreads), 0, (hipStream_t)stream, m, params,
                       param_stride, temp, n_species, n_h2, radius, flags);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}
