// Emission (eclipse) geometry of the forward model (Sec. 3 and Sec. 4: transit's emission
// spectra; Sec. 6: the intensity spectra of the eclipse-geometry tests). After the same
// record preparation as the transit geometry, one workgroup takes 256 wavenumbers of one
// sample (one per lane) and walks the layers from the top: the extinction e_l from the
// tables (as in the transit kernel's first phase), the vertical optical depth by the
// trapezoid in height, and the emergent intensity along the normal with the Planck function
// as source (the two layers' mean between them, the deepest layer radiating from below):
//   I = B(T_0) e^{-tau_0} + sum_l (B(T_l) + B(T_{l+1}))/2 (e^{-tau_{l+1}} - e^{-tau_l}).
// The per-layer record fields are the same for every lane (scalar loads); the table rows are
// read along nu (coalesced). Optical depth, source and intensity are in double.
#include "bm_forward.h"

namespace bm {

constexpr int kEmThreads = 256;
constexpr double kPlanckC1 = 2.0 * 6.62607015e-27 * 2.99792458e10 * 2.99792458e10;  // 2 h c^2

template <typename T, int kS, bool kCia>
__global__ void __launch_bounds__(kEmThreads)
    k_emission(ModelDev m, const char* __restrict__ ws, size_t rec_bytes, const int32_t* __restrict__ active,
               double* __restrict__ out) {
    const int s_in = blockIdx.y;
    if (active && !active[s_in]) return;  // sample not requested in this call
    const int L = m.L, Nnu = m.Nnu;
    const RecordView<T> rec(const_cast<char*>(ws) + (size_t)s_in * rec_bytes, kS, L);
    const int nu = blockIdx.x * kEmThreads + threadIdx.x;
    const bool valid = nu < Nnu;
    const int nuc = valid ? nu : Nnu - 1;
    double* o = out + (size_t)s_in * Nnu;
    if (rec.hdr->flags & BM_FLAG_RADIUS) {
        if (valid) o[nu] = __builtin_nan("");
        return;
    }
    const double nuv = m.nu_start + m.dnu * nuc;
    const double b_num = kPlanckC1 * nuv * nuv * nuv;
    const double c2nu = kC2 * nuv;
    const T sray = m.rayleigh ? (T)rayleigh_h2_xsec(nuv) : T(0);
    const T* __restrict__ sig = static_cast<const T*>(m.sigma);
    const size_t t_stride = (size_t)L * Nnu;
    const size_t s_stride = (size_t)m.NT * t_stride;
    auto extinction = [&](int l) -> double {
        const T* p = sig + (size_t)rec.kidx[l] * t_stride + (size_t)l * Nnu + nuc;
        const T w = rec.w[l];
        T e = T(0);
#pragma unroll
        for (int i = 0; i < kS; ++i) {
            const T s0 = p[i * s_stride], s1 = p[i * s_stride + t_stride];
            e = fma(rec.afac[i * L + l], fma(w, s1 - s0, s0), e);
        }
        if constexpr (kCia) {
            const double* c = m.cia + (size_t)rec.kcidx[l] * Nnu + nuc;
            e += (T)(rec.bfac[l] * fma(rec.wc[l], c[Nnu] - c[0], c[0]));
        }
        if (m.rayleigh) e = fma(rec.rfac[l], sray, e);
        return (double)e;
    };
    auto planck = [&](int l) -> double { return b_num / expm1(c2nu / rec.tl[l]); };
    double e_up = extinction(L - 1);
    double tau = 0.0, att_up = 1.0, b_up = planck(L - 1), inten = 0.0;
    for (int l = L - 2; l >= 0; --l) {
        const double e = extinction(l);
        tau += (rec.rl[l + 1] - rec.rl[l]) * 0.5 * (e + e_up);
        const double att = exp(-tau);
        const double b = planck(l);
        inten += 0.5 * (b + b_up) * (att_up - att);
        e_up = e;
        att_up = att;
        b_up = b;
    }
    inten += b_up * att_up;  // the deepest layer, radiating from below
    if (valid) o[nu] = inten;
}

template <typename T, bool kCia>
static void emission_dispatch(int S, dim3 grid, hipStream_t st, const ModelDev& m, const char* ws, size_t rb,
                              const int32_t* act, double* out) {
    switch (S) {
#define BM_EM_CASE(NS) \
    case NS: hipLaunchKernelGGL((k_emission<T, NS, kCia>), grid, dim3(kEmThreads), 0, st, m, ws, rb, act, out); break;
        BM_EM_CASE(1) BM_EM_CASE(2) BM_EM_CASE(3) BM_EM_CASE(4) BM_EM_CASE(5) BM_EM_CASE(6) BM_EM_CASE(7) BM_EM_CASE(8)
#undef BM_EM_CASE
        default: break;
    }
}

template <typename T>
int launch_k_emission(const LaunchPlan& lp, int si, char* ws, const int32_t* act, double* out, hipStream_t st) {
    const Segment& sg = lp.seg[si];
    const ModelDev& m = lp.model[sg.model];
    if (m.S < 1 || m.S > BM_MAX_SPECIES) return BM_ESHAPE;
    const dim3 grid((m.Nnu + kEmThreads - 1) / kEmThreads, sg.count);
    const int32_t* a = act ? act + sg.first : nullptr;
    if (m.NTc > 0)
        emission_dispatch<T, true>(m.S, grid, st, m, ws + sg.ws_off, sg.rec_bytes, a, out + sg.depth_off);
    else
        emission_dispatch<T, false>(m.S, grid, st, m, ws + sg.ws_off, sg.rec_bytes, a, out + sg.depth_off);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

template int launch_k_emission<float>(const LaunchPlan&, int, char*, const int32_t*, double*, hipStream_t);
template int launch_k_emission<double>(const LaunchPlan&, int, char*, const int32_t*, double*, hipStream_t);

}  // namespace bm
