// Steps a1-a2 of the forward model on the GPU: parameters -> per-layer temperature,
// composition, number densities and hydrostatic radii (Sec. 3 profile generator;
// Sec. 6.2 radius at the reference pressure; Sec. 6.3 / Sec. 7 parameterisation),
// plus the per-sample record consumed by the fused forward kernel: T-interpolation
// brackets, density factors, FP64 chord weights rounded once to the compute type,
// and the impact-parameter quadrature coefficients.
#include "bm_forward.h"

namespace bm {

// One workgroup (kAtmThreads threads) evaluates one sample. Layer l is owned by
// thread l (L <= BM_MAX_LAYERS = kAtmThreads). Results are left in shared memory.
struct AtmShared {
    double temp[BM_MAX_LAYERS];
    double radius[BM_MAX_LAYERS];
    double ndens[BM_MAX_LAYERS];
    double scan[BM_MAX_LAYERS];
    double x[BM_MAX_SPECIES];
    double x_h2;
    double mu;
    int flags;
};

__device__ void atm_compute(const ModelDev& m, const double* __restrict__ theta, AtmShared& sh) {
    const int tid = threadIdx.x;
    const int L = m.L;
    const int ntp = (m.tp_mode == BM_TP_ISOTHERMAL) ? 1 : 5;
    if (tid == 0) {
        int flags = 0;
        const int np = ntp + m.S + 1;
        for (int i = 0; i < np; ++i)
            if (!isfinite(theta[i])) flags |= BM_FLAG_NONFINITE;
        double total = 0.0;
        for (int i = 0; i < m.S; ++i) {
            sh.x[i] = pow(10.0, theta[ntp + i]);
            total += sh.x[i];
        }
        if (total >= 1.0) flags |= BM_FLAG_SUM_X;
        double fill = 1.0 - total;
        if (fill < 0.0) fill = 0.0;
        double x_h2 = m.pl.h2_frac * fill;
        double x_he = (1.0 - m.pl.h2_frac) * fill;
        double mu = 0.0;
        for (int i = 0; i < m.S; ++i) mu += sh.x[i] * m.mass[i];
        mu += x_h2 * m.pl.m_h2_amu + x_he * m.pl.m_he_amu;
        sh.x_h2 = x_h2;
        sh.mu = mu;
        sh.flags = flags;
    }
    // temperature and number density per layer
    if (tid < L) {
        double p = m.p_bar[tid];
        double t = (m.tp_mode == BM_TP_ISOTHERMAL) ? theta[0] : line2013_temperature(p, theta, m.pl);
        sh.temp[tid] = t;
        sh.ndens[tid] = p * kBar / (kBoltz * t);
    }
    __syncthreads();
    if (tid < L && !(isfinite(sh.temp[tid]) && sh.temp[tid] > 0.0))
        atomicOr(&sh.flags, BM_FLAG_NONFINITE);
    // hydrostatic radii: 1/r_l = 1/R_ref + k_B/(GM mu m_u) (I_l - I_ref), with I the
    // exact integral of the piecewise-linear (in ln p) temperature from layer 0.
    // segment integrals, then an inclusive Hillis-Steele scan over layers
    if (tid < L) {
        double seg = 0.0;
        if (tid > 0) {
            double a = log(m.p_bar[tid - 1]), b = log(m.p_bar[tid]);
            seg = (b - a) * 0.5 * (sh.temp[tid - 1] + sh.temp[tid]);
        }
        sh.scan[tid] = seg;
    }
    __syncthreads();
    for (int off = 1; off < L; off <<= 1) {
        double v = 0.0;
        if (tid < L && tid >= off) v = sh.scan[tid - off];
        __syncthreads();
        if (tid < L && tid >= off) sh.scan[tid] += v;
        __syncthreads();
    }
    if (tid < L) {
        // layer m with ln p_m >= ln p_ref > ln p_{m+1}; pressures decrease with l
        const double lnref = log(m.pl.p_ref_bar);
        int mref = 0;
        for (int i = 0; i < L - 1; ++i)
            if (log(m.p_bar[i]) >= lnref) mref = i;
        double la = log(m.p_bar[mref]), lb = log(m.p_bar[mref + 1]);
        double tref = sh.temp[mref] + (sh.temp[mref + 1] - sh.temp[mref]) * (lnref - la) / (lb - la);
        double iref = sh.scan[mref] + (lnref - la) * 0.5 * (sh.temp[mref] + tref);
        double gm = m.pl.g_nom * m.pl.r_nom_cm * m.pl.r_nom_cm;
        double coef = kBoltz / (gm * sh.mu * kAmu);
        double rref = theta[ntp + m.S] * kRJup;
        double inv_r = 1.0 / rref + coef * (sh.scan[tid] - iref);
        if (!(inv_r > 0.0)) {
            atomicOr(&sh.flags, BM_FLAG_RADIUS);
            sh.radius[tid] = NAN;
        } else {
            sh.radius[tid] = 1.0 / inv_r;
        }
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kAtmThreads) k_atmosphere(ModelDev m, const double* __restrict__ params,
                                                            int stride, double* temp, double* n_species,
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
        for (int i = 0; i < m.S; ++i)
            n_species[((size_t)b * m.S + i) * L + tid] = sh.x[i] * sh.ndens[tid];
    }
    if (tid == 0) flags[b] = sh.flags;
}

// Per-sample record for the fused forward kernel.
template <typename T>
__global__ void __launch_bounds__(kAtmThreads) k_atm_prep(LaunchPlan plan, const double* __restrict__ params,
                                                          int stride, char* __restrict__ ws,
                                                          int32_t* __restrict__ flags_out) {
    __shared__ AtmShared sh;
    const int b = blockIdx.x;
    const int si = plan.segment_of_sample(b);
    const Segment& sg = plan.seg[si];
    const ModelDev& m = plan.model[sg.model];
    atm_compute(m, params + (size_t)b * stride, sh);
    const int tid = threadIdx.x;
    const int L = m.L;
    RecordView<T> rec(ws + sg.ws_off + (size_t)(b - sg.first) * sg.rec_bytes, m.S, L);

    int flags_local = 0;
    if (tid < L) {
        int k, kc = 0;
        double w, wc = 0.0;
        double t = sh.temp[tid];
        if (interp_bracket(m.temp, m.NT, t, &k, &w)) flags_local |= BM_FLAG_T_CLAMP;
        if (m.NTc > 0 && interp_bracket(m.temp_cia, m.NTc, t, &kc, &wc)) flags_local |= BM_FLAG_T_CLAMP;
        rec.kidx[tid] = k;
        rec.kcidx[tid] = kc;
        rec.w[tid] = (T)w;
        rec.wc[tid] = (T)wc;
        double nh2 = sh.x_h2 * sh.ndens[tid];
        rec.bfac[tid] = (T)(nh2 * nh2);
        for (int i = 0; i < m.S; ++i) rec.afac[i * L + tid] = (T)(sh.x[i] * sh.ndens[tid]);
        // impact-parameter quadrature weight of f_j (trapezoid in b)
        const double* r = sh.radius;
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
    // chord weights, blocked [nb][L][kRows]: W[j][l] = [l <= L-2](s_{j,l+1} - s_{j,l})
    //   + [l >= j+1](s_{j,l} - s_{j,l-1}) for l >= j and j <= L-2, zero otherwise
    const int nb = rec.nb;
    const double* r = sh.radius;
    for (int idx = tid; idx < nb * L * kRows; idx += kAtmThreads) {
        const int rr = idx % kRows;
        const int l = (idx / kRows) % L;
        const int blk = idx / (kRows * L);
        const int j = blk * kRows + rr;
        double wv = 0.0;
        if (j <= L - 2 && l >= j) {
            double s_l = (l == j) ? 0.0 : half_chord(r[l], r[j]);
            if (l <= L - 2) wv += half_chord(r[l + 1], r[j]) - s_l;
            if (l >= j + 1) wv += s_l - ((l - 1 == j) ? 0.0 : half_chord(r[l - 1], r[j]));
        }
        rec.wb[idx] = (T)wv;
    }
    __syncthreads();
    if (tid == 0) {
        rec.hdr->base = r[0] * r[0];
        rec.hdr->rs2 = m.pl.rs_cm * m.pl.rs_cm;
        rec.hdr->flags = sh.flags;
        flags_out[b] = sh.flags;
    }
}

template __global__ void k_atm_prep<float>(LaunchPlan, const double*, int, char*, int32_t*);
template __global__ void k_atm_prep<double>(LaunchPlan, const double*, int, char*, int32_t*);

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
