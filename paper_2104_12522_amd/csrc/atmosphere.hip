// Steps a1-a2 of the forward model on the GPU: parameters -> per-layer temperature,
// composition, number densities and hydrostatic radii (Sec. 3 profile generator;
// Sec. 6.2 radius at the reference pressure; Sec. 6.3 / Sec. 7 parameterisation),
// plus the per-sample record consumed by the fused forward kernel: T-interpolation
// brackets, density factors, FP64 chord weights rounded once to the compute type
// (laid out as matrix-core A fragments in FP32), and the impact-parameter weights.
#include "bm_forward.h"

namespace bm {

// One workgroup evaluates one sample; layer l is owned by thread l (L <= BM_MAX_LAYERS).
struct AtmShared {
    double tgrid[BM_MAX_TEMPS];
    double tgrid_cia[BM_MAX_TEMPS];
    double temp[BM_MAX_LAYERS];
    double radius[BM_MAX_LAYERS];
    double ndens[BM_MAX_LAYERS];
    double lnp[BM_MAX_LAYERS];
    double scan[BM_MAX_LAYERS];
    double wave_tot[kAtmThreads / kWave];
    double x[BM_MAX_SPECIES];
    double theta[5 + BM_MAX_SPECIES + 2];
    Line2013Consts tp;
    double x_h2;
    double mu;
    double iref;
    int flags;
    int jcloud;  // largest layer at or below the cloud top (-1: none or no cloud deck)
};

__device__ void atm_compute(const ModelDev& m, const double* __restrict__ theta_g, AtmShared& sh) {
    const int tid = threadIdx.x;
    const int L = m.L;
    const int ntp = (m.tp_mode == BM_TP_ISOTHERMAL) ? 1 : 5;
    const int np = ntp + m.S + 1 + m.cloud;
    // parameters, temperature grids, layer pressures: one round of loads
    if (tid < np) sh.theta[tid] = theta_g[tid];
    if (tid < m.NT && m.temp) sh.tgrid[tid] = m.temp[tid];
    if (tid < m.NTc && m.temp_cia) sh.tgrid_cia[tid] = m.temp_cia[tid];
    if (tid == 0) sh.jcloud = -1;
    // with L <= 128 the Line-2013 profile's two xi() terms of layer l are evaluated by
    // threads l and l + 128 (a dependent chain half as long)
    const bool split = (m.tp_mode == BM_TP_LINE2013) && (2 * L <= kAtmThreads);
    const int lay = split ? (tid & (kAtmThreads / 2 - 1)) : tid;
    const bool upper = split && tid >= kAtmThreads / 2;
    double p = 0.0;
    if (lay < L && (split || tid < L)) p = m.p_bar[lay];
    __syncthreads();
    const double* theta = sh.theta;
    // per-sample constants, each on its own thread
    if (tid < m.S) sh.x[tid] = pow10_(theta[ntp + tid]);
    if (m.tp_mode == BM_TP_LINE2013 && tid >= 32 && tid < 36) line2013_consts_part(theta, m.pl, tid - 32, &sh.tp);
    // gray cloud deck: the largest layer with p_l >= p_cloud (any layer order)
    if (m.cloud && tid < L && p >= pow10_(theta[np - 1])) atomicMax(&sh.jcloud, tid);
    __syncthreads();
    // totals, mean molecular mass and flags on the last thread, which has no layer of its
    // own in the split profile evaluation below
    if (tid == kAtmThreads - 1) {
        int flags = 0;
        for (int i = 0; i < np; ++i)
            if (!isfinite(theta[i])) flags |= BM_FLAG_NONFINITE;
        double total = 0.0;
        for (int i = 0; i < m.S; ++i) total += sh.x[i];
        if (total >= 1.0) flags |= BM_FLAG_SUM_X;
        double fill = 1.0 - total;
        if (fill < 0.0) fill = 0.0;
        const double x_h2 = m.pl.h2_frac * fill;
        const double x_he = (1.0 - m.pl.h2_frac) * fill;
        double mu = 0.0;
        for (int i = 0; i < m.S; ++i) mu += sh.x[i] * m.mass[i];
        mu += x_h2 * m.pl.m_h2_amu + x_he * m.pl.m_he_amu;
        sh.x_h2 = x_h2;
        sh.mu = mu;
        sh.flags = flags;
    }
    // temperature, number density and ln p per layer
    if (split) {
        const double tau = line2013_tau(p, sh.tp);
        double xi = 0.0;
        if (lay < L) xi = line2013_xi(upper ? sh.tp.g2 : sh.tp.g1, tau);
        if (upper && lay < L) sh.scan[lay] = xi;  // scratch until the radius scan
        if (!upper && lay < L) sh.lnp[lay] = log(p);
        __syncthreads();
        if (tid < L) {
            const double t = line2013_temperature_xi(tau, xi, sh.scan[tid], sh.tp);
            sh.temp[tid] = t;
            sh.ndens[tid] = p * kBar / (kBoltz * t);
        }
    } else if (tid < L) {
        const double t = (m.tp_mode == BM_TP_ISOTHERMAL) ? theta[0] : line2013_temperature_c(p, sh.tp);
        sh.temp[tid] = t;
        sh.ndens[tid] = p * kBar / (kBoltz * t);
        sh.lnp[tid] = log(p);
    }
    __syncthreads();
    if (tid < L && !(isfinite(sh.temp[tid]) && sh.temp[tid] > 0.0)) atomicOr(&sh.flags, BM_FLAG_NONFINITE);
    // hydrostatic radii: 1/r_l = 1/R_ref + k_B/(GM mu m_u) (I_l - I_ref), with I the
    // exact integral of the piecewise-linear (in ln p) temperature from layer 0:
    // segment integrals, an inclusive scan within each wave (shuffles), then each wave
    // adds the totals of the waves before it
    {
        double v = (tid > 0 && tid < L) ? (sh.lnp[tid] - sh.lnp[tid - 1]) * 0.5 * (sh.temp[tid - 1] + sh.temp[tid]) : 0.0;
        const int lane = tid & (kWave - 1), w = tid / kWave;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const double u = __shfl_up(v, off, kWave);
            if (lane >= off) v += u;
        }
        if (lane == kWave - 1) sh.wave_tot[w] = v;
        __syncthreads();
        for (int q = 0; q < w; ++q) v += sh.wave_tot[q];
        if (tid < L) sh.scan[tid] = v;
    }
    __syncthreads();
    // the layer m with ln p_m >= ln p_ref > ln p_{m+1} (pressures decrease with l; m is
    // clamped to [0, L-2], i.e. linear extrapolation outside the grid)
    const double lnref = log(m.pl.p_ref_bar);
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
    __syncthreads();
    if (tid < L) {
        const double gm = m.pl.g_nom * m.pl.r_nom_cm * m.pl.r_nom_cm;
        const double coef = kBoltz / (gm * sh.mu * kAmu);
        const double rref = sh.theta[ntp + m.S] * kRJup;
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
    const int b = blockIdx.x;
    atm_compute(m, params + (size_t)b * stride, sh);
    const int tid = threadIdx.x;
    const int L = m.L;
    if (tid < L) {
        temp[(size_t)b * L + tid] = sh.temp[tid];
        radius[(size_t)b * L + tid] = sh.radius[tid];
        n_h2[(size_t)b * L + tid] = sh.x_h2 * sh.ndens[tid];
        for (int i = 0; i < m.S; ++i) n_species[((size_t)b * m.S + i) * L + tid] = sh.x[i] * sh.ndens[tid];
    }
    if (tid == 0) flags[b] = sh.flags;
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
template <typename T>
__global__ void __launch_bounds__(kAtmThreads)
    k_atm_prep(LaunchPlan plan, const double* __restrict__ params, int stride, const int32_t* __restrict__ active,
               char* __restrict__ ws, int32_t* __restrict__ flags_out) {
    __shared__ AtmShared sh;
    const int b = blockIdx.x;
    if (active && !active[b]) return;  // sample not requested in this call
    const int slice = blockIdx.y, n_slices = gridDim.y;
    const int si = plan.segment_of_sample(b);
    const Segment& sg = plan.seg[si];
    const ModelDev& m = plan.model[sg.model];
    atm_compute(m, params + (size_t)b * stride, sh);
    const int tid = threadIdx.x;
    const int L = m.L;
    RecordView<T> rec(ws + sg.ws_off + (size_t)(b - sg.first) * sg.rec_bytes, m.S, L);
    const double* r = sh.radius;

    if (slice == 0) {
        int flags_local = 0;
        if (tid < L) {
            int k, kc = 0;
            double w, wc = 0.0;
            const double t = sh.temp[tid];
            if (interp_bracket(sh.tgrid, m.NT, t, &k, &w)) flags_local |= BM_FLAG_T_CLAMP;
            if (m.NTc > 0 && interp_bracket(sh.tgrid_cia, m.NTc, t, &kc, &wc)) flags_local |= BM_FLAG_T_CLAMP;
            rec.kidx[tid] = k;
            rec.kcidx[tid] = kc;
            rec.w[tid] = (T)w;
            rec.wc[tid] = wc;
            const double nh2 = sh.x_h2 * sh.ndens[tid];
            rec.bfac[tid] = nh2 * nh2;
            rec.rfac[tid] = (T)nh2;
            for (int i = 0; i < m.S; ++i) rec.afac[i * L + tid] = (T)(sh.x[i] * sh.ndens[tid]);
            // impact-parameter quadrature weight of f_j (trapezoid in b)
            double c;
            if (tid == 0)
                c = (r[1] - r[0]) * r[0];
            else if (tid == L - 1)
                c = (r[L - 1] - r[L - 2]) * r[L - 1];
            else
                c = r[tid] * (r[tid + 1] - r[tid - 1]);
            rec.cw[tid] = c;
        }
        if (flags_local) atomicOr(&sh.flags, flags_local);
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
}

template __global__ void k_atm_prep<float>(LaunchPlan, const double*, int, const int32_t*, char*, int32_t*);
template __global__ void k_atm_prep<double>(LaunchPlan, const double*, int, const int32_t*, char*, int32_t*);

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
