// Differential-evolution MCMC with a past-state archive and snooker moves (DEMCzs) and
// two-stage delayed acceptance, on the GPU. BART samples its posterior with MC3's
// differential-evolution samplers (Sec. 3, Sec. 4 item 10, Sec. 5: DEMC of ter Braak 2006
// and the archive-based DEMCzs of ter Braak & Vrugt 2008); this file implements the
// archive proposals for a whole generation of chains at once, so that every chain's
// forward model of a generation runs in one batched launch.
//
// DE move (ter Braak & Vrugt 2008): y_i = x_i + gamma (z_r1 - z_r2) + e,
//   r1 != r2 drawn uniformly from the archive, gamma = 2.38 / sqrt(2 d) except every
//   10th generation (gamma = 1, mode jumping), e ~ N(0, (eps_scale * width)^2) per
//   parameter. Symmetric given the archive.
// Snooker move (same paper), taken with probability p_snooker: a third archive row z
//   distinct from r1 and r2; u = (x - z) / |x - z|; y = x + gamma_s ((z_r1 - z_r2) . u) u
//   with gamma_s ~ U[1.2, 2.2); Hastings factor (|y - z| / |x - z|)^(d - 1).
// Acceptance: Metropolis-Hastings with log pi = -chi^2 / 2 inside the uniform prior box.
// Delayed acceptance (Christen & Fox 2005): stage 1 accepts with
//   min(1, exp(lp*_y - lp*_x + log q)) using a cheap surrogate; only stage-1 survivors run
//   the exact forward model, and stage 2 accepts with min(1, exp((lp_y - lp_x) - (lp*_y -
//   lp*_x))) (the proposal factor cancels), which leaves the exact posterior invariant.
//
// Random numbers: a counter-based generator, SplitMix64 (Steele, Lea & Flood 2014):
// the k-th output of the stream with seed s is mix(s + (k + 1) * 0x9E3779B97F4A7C15),
// mix(z) = z ^ (z >> 30) * 0xBF58476D1CE4E5B9, ^ (>> 27) * 0x94D049BB133111EB, ^ (>> 31).
// Draw k of chain c in generation g uses counter ((g * C + c) * kSlots + slot). Normals
// by Box-Muller from two uniforms.
#include "bm_internal.h"

#include <cmath>

// Sampler arithmetic is specified operation by operation (proposals, prior draws): no
// fused multiply-adds in this file, so every rounding is the one written.
#pragma clang fp contract(off)

namespace bm {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr int kSlots = 64;           // random draws reserved per (generation, chain)
constexpr int kSlotR1 = 0, kSlotR2 = 1, kSlotU = 2, kSlotU1 = 3, kSlotNormal = 8;
constexpr int kSlotMove = 4, kSlotZ = 5, kSlotGammaS = 6;  // snooker: choice, row z, gamma_s
constexpr int kMaxParams = (kSlots - kSlotNormal) / 2;     // two normal uniforms per parameter

__host__ __device__ inline uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * kGolden;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// uniform double in [0, 1): the top 53 bits
__host__ __device__ inline double u01(uint64_t seed, uint64_t k) {
    return (double)(splitmix64(seed, k) >> 11) * 0x1.0p-53;
}

__device__ inline uint64_t counter(int64_t g, int c, int C, int slot) {
    return ((uint64_t)g * (uint64_t)C + (uint64_t)c) * kSlots + (uint64_t)slot;
}

// standard normal number j of (g, c): Box-Muller on uniforms (2j, 2j+1) of the normal slots
__device__ inline double normal_draw(uint64_t seed, int64_t g, int c, int C, int j) {
    const double u1 = u01(seed, counter(g, c, C, kSlotNormal + 2 * j));
    const double u2 = u01(seed, counter(g, c, C, kSlotNormal + 2 * j + 1));
    const double rad = sqrt(-2.0 * log(1.0 - u1));  // 1 - u1 in (0, 1]
    return rad * cos(6.283185307179586476925 * u2);
}

// counters: [0] generation, [1] archive size
// One thread per (chain, parameter): the DE move's components, each with its own normal draw,
// in parallel; the snooker move (sums over the parameters) by each chain's parameter-0
// thread. Every element is computed with the same operations either way.
__global__ void k_demcz_propose(bm_demcz s, double gamma_de) {
    const int d = s.n_params;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = t / d, p = t - c * d;
    if (c >= s.n_chains) return;
    const int64_t g = s.counters[0];
    const int M = s.counters[1];
    // two distinct archive members
    int r1 = (int)(u01(s.seed, counter(g, c, s.n_chains, kSlotR1)) * M);
    int r2 = (int)(u01(s.seed, counter(g, c, s.n_chains, kSlotR2)) * (M - 1));
    if (r1 >= M) r1 = M - 1;
    if (r2 >= M - 1) r2 = M - 2;
    if (r2 >= r1) r2 += 1;
    const double* x = s.x + (size_t)c * d;
    double* y = s.prop + (size_t)c * d;
    const bool snooker = s.p_snooker > 0.0 && M >= 3 && u01(s.seed, counter(g, c, s.n_chains, kSlotMove)) < s.p_snooker;
    if (!snooker) {
        const double gamma = (g % 10 == 9) ? 1.0 : gamma_de;
        const double width = s.hi[p] - s.lo[p];
        // written operation by operation; contraction is off in this file
        const double e = (s.eps_scale * width) * normal_draw(s.seed, g, c, s.n_chains, p);
        const double diff = s.z[(size_t)r1 * d + p] - s.z[(size_t)r2 * d + p];
        const double step = gamma * diff;
        y[p] = (x[p] + step) + e;
        if (p == 0 && s.log_q) s.log_q[c] = 0.0;
        return;
    }
    if (p != 0) return;
    // snooker: a third row, uniform over the M - 2 rows other than r1 and r2
    int rz = (int)(u01(s.seed, counter(g, c, s.n_chains, kSlotZ)) * (M - 2));
    if (rz >= M - 2) rz = M - 3;
    const int ra = min(r1, r2), rb = max(r1, r2);
    if (rz >= ra) rz += 1;
    if (rz >= rb) rz += 1;
    const double* zz = s.z + (size_t)rz * d;
    const double* z1 = s.z + (size_t)r1 * d;
    const double* z2 = s.z + (size_t)r2 * d;
    double nn = 0.0, dot = 0.0;
    for (int q = 0; q < d; ++q) {
        const double e = x[q] - zz[q];
        nn = nn + e * e;
        dot = dot + (z1[q] - z2[q]) * e;
    }
    double lq = -INFINITY;  // x on z: no line, no move
    if (nn > 0.0) {
        const double gamma_s = 1.2 + u01(s.seed, counter(g, c, s.n_chains, kSlotGammaS));
        const double coef = gamma_s * (dot / nn);
        double n2 = 0.0;
        for (int q = 0; q < d; ++q) {
            y[q] = x[q] + coef * (x[q] - zz[q]);
            const double f = y[q] - zz[q];
            n2 = n2 + f * f;
        }
        const int k = s.n_free > 0 ? s.n_free : d;  // the dimension the chains move in
        if (n2 > 0.0) lq = (0.5 * (k - 1)) * (log(n2) - log(nn));
    } else {
        for (int q = 0; q < d; ++q) y[q] = x[q];
    }
    s.log_q[c] = lq;
}

__device__ inline bool in_box(const bm_demcz& s, const double* y) {
    for (int p = 0; p < s.n_params; ++p)
        if (!(y[p] >= s.lo[p] && y[p] <= s.hi[p])) return false;
    return true;
}

// log posterior of a proposal from its chi^2 and flags (-inf outside the box or flagged)
__device__ inline double log_post(const bm_demcz& s, const double* y, double chi2, int flags) {
    if (!in_box(s, y) || flags != 0 || !isfinite(chi2)) return -INFINITY;
    return -0.5 * chi2;
}

// plain Metropolis acceptance, then history / archive bookkeeping
__global__ void k_demcz_accept(bm_demcz s, const double* __restrict__ chi2, const int32_t* __restrict__ flags,
                               const double* __restrict__ chi2_surr, const int32_t* __restrict__ active,
                               int mode) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int C = s.n_chains, d = s.n_params;
    const int64_t g = s.counters[0];
    const int M = s.counters[1];
    if (c < C) {
        const double* y = s.prop + (size_t)c * d;
        bool take = false;
        if (mode == 0) {
            const double lpy = log_post(s, y, chi2[c], flags ? flags[c] : 0);
            const double u = u01(s.seed, counter(g, c, C, kSlotU));
            const double lq = s.log_q ? s.log_q[c] : 0.0;
            take = isfinite(lpy) && log(u) < (lpy - s.lp[c]) + lq;
            if (take) s.lp[c] = lpy;
        } else {
            // delayed acceptance, stage 2: only stage-1 survivors were evaluated
            if (active[c]) {
                s.n_accept[2 * c] += 1;
                const double lpy = log_post(s, y, chi2[c], flags ? flags[c] : 0);
                const double lsy = -0.5 * chi2_surr[c];
                const double u = u01(s.seed, counter(g, c, C, kSlotU));
                take = isfinite(lpy) && log(u) < (lpy - s.lp[c]) - (lsy - s.lp_surr[c]);
                if (take) {
                    s.lp[c] = lpy;
                    s.lp_surr[c] = lsy;
                }
            }
        }
        if (take) {
            s.n_accept[2 * c + 1] += 1;
            for (int p = 0; p < d; ++p) s.x[(size_t)c * d + p] = y[p];
        }
        if (s.history && g < s.hist_cap)
            for (int p = 0; p < d; ++p) s.history[((size_t)g * C + c) * d + p] = s.x[(size_t)c * d + p];
        // archive: append every `thin` generations while there is room
        if ((g + 1) % s.thin == 0 && M + C <= s.z_cap)
            for (int p = 0; p < d; ++p) s.z[(size_t)(M + c) * d + p] = s.x[(size_t)c * d + p];
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // single-block launch: every chain's bookkeeping above has completed
        if ((g + 1) % s.thin == 0 && M + C <= s.z_cap) s.counters[1] = M + C;
        s.counters[0] = g + 1;
    }
}

// delayed acceptance, stage 1: screen proposals with the surrogate's chi^2
__global__ void k_da_screen(bm_demcz s, const double* __restrict__ chi2_surr, int32_t* __restrict__ active) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= s.n_chains) return;
    const double* y = s.prop + (size_t)c * s.n_params;
    const int64_t g = s.counters[0];
    int a = 0;
    if (in_box(s, y) && isfinite(chi2_surr[c])) {
        const double u = u01(s.seed, counter(g, c, s.n_chains, kSlotU1));
        const double lq = s.log_q ? s.log_q[c] : 0.0;
        a = log(u) < ((-0.5 * chi2_surr[c]) - s.lp_surr[c]) + lq;
    }
    active[c] = a;
}

// chains start at uniform prior draws (generation counter -1, i.e. before the first
// generation), the archive with z_init further prior draws
__global__ void k_demcz_init(bm_demcz s, int z_init) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int d = s.n_params;
    const int total = z_init + s.n_chains;
    if (i < total) {
        for (int p = 0; p < d; ++p) {
            const double u = u01(s.seed ^ 0xA5A5A5A5A5A5A5A5ull, (uint64_t)i * kSlots + p);
            const double v = s.lo[p] + (s.hi[p] - s.lo[p]) * u;
            if (i < z_init)
                s.z[(size_t)i * d + p] = v;
            else
                s.x[(size_t)(i - z_init) * d + p] = v;
        }
        if (i >= z_init) {
            const int c = i - z_init;
            s.n_accept[2 * c] = 0;
            s.n_accept[2 * c + 1] = 0;
        }
    }
    if (i == 0) {
        s.counters[0] = 0;
        s.counters[1] = z_init;
    }
}

// log posterior of the current states from their chi^2 (after the initial forward model)
__global__ void k_demcz_set_lp(bm_demcz s, const double* __restrict__ chi2, const int32_t* __restrict__ flags,
                               const double* __restrict__ chi2_surr) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= s.n_chains) return;
    const double* x = s.x + (size_t)c * s.n_params;
    if (chi2) s.lp[c] = log_post(s, x, chi2[c], flags ? flags[c] : 0);
    if (chi2_surr && s.lp_surr) s.lp_surr[c] = -0.5 * chi2_surr[c];
}

}  // namespace bm

using namespace bm;

static int check_demcz(const bm_demcz* s) {
    if (!s || !s->x || !s->lp || !s->prop || !s->z || !s->counters || !s->n_accept || !s->lo || !s->hi)
        return BM_EINVAL;
    if (s->n_chains < 1 || s->n_chains > 1024 || s->n_params < 1 || s->n_params > kMaxParams) return BM_ESHAPE;
    if (s->thin < 1 || s->z_cap < 2) return BM_ESHAPE;
    if (!(s->eps_scale >= 0.0)) return BM_EINVAL;
    if (!(s->p_snooker >= 0.0 && s->p_snooker <= 1.0)) return BM_EINVAL;
    if (!(s->gamma_scale >= 0.0 && s->gamma_scale <= 4.0)) return BM_EINVAL;
    if (s->n_free < 0 || s->n_free > s->n_params) return BM_ESHAPE;
    if (s->p_snooker > 0.0 && !s->log_q) return BM_EINVAL;
    return BM_OK;
}

extern "C" int bm_demcz_init(const bm_demcz* s, int z_init, void* stream) {
    int st = check_demcz(s);
    if (st != BM_OK) return st;
    if (z_init < 2 || z_init > s->z_cap) return BM_ESHAPE;
    const int total = z_init + s->n_chains;
    hipLaunchKernelGGL(k_demcz_init, dim3((total + 255) / 256), dim3(256), 0, (hipStream_t)stream, *s, z_init);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

extern "C" int bm_demcz_set_lp(const bm_demcz* s, const double* chi2, const int32_t* flags, const double* chi2_surr,
                               void* stream) {
    int st = check_demcz(s);
    if (st != BM_OK) return st;
    if (!chi2 && !chi2_surr) return BM_EINVAL;
    if (chi2_surr && !s->lp_surr) return BM_EINVAL;
    hipLaunchKernelGGL(k_demcz_set_lp, dim3((s->n_chains + 255) / 256), dim3(256), 0, (hipStream_t)stream, *s, chi2,
                       flags, chi2_surr);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

extern "C" int bm_demcz_propose(const bm_demcz* s, void* stream) {
    int st = check_demcz(s);
    if (st != BM_OK) return st;
    // gamma = gamma_scale (2.38 / sqrt(2 k)), k free parameters (correctly rounded host
    // arithmetic)
    const double scale = s->gamma_scale > 0.0 ? s->gamma_scale : 1.0;
    const int k = s->n_free > 0 ? s->n_free : s->n_params;
    const double gamma_de = scale * (2.38 / std::sqrt(2.0 * k));
    const int64_t n_threads = (int64_t)s->n_chains * s->n_params;
    hipLaunchKernelGGL(k_demcz_propose, dim3((unsigned)((n_threads + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       *s, gamma_de);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

extern "C" int bm_demcz_accept(const bm_demcz* s, const double* chi2, const int32_t* flags, void* stream) {
    int st = check_demcz(s);
    if (st != BM_OK) return st;
    if (!chi2) return BM_EINVAL;
    hipLaunchKernelGGL(k_demcz_accept, dim3(1), dim3(1024), 0, (hipStream_t)stream, *s, chi2, flags,
                       (const double*)nullptr, (const int32_t*)nullptr, 0);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

extern "C" int bm_da_screen(const bm_demcz* s, const double* chi2_surr, int32_t* active, void* stream) {
    int st = check_demcz(s);
    if (st != BM_OK) return st;
    if (!chi2_surr || !active || !s->lp_surr) return BM_EINVAL;
    hipLaunchKernelGGL(k_da_screen, dim3((s->n_chains + 255) / 256), dim3(256), 0, (hipStream_t)stream, *s, chi2_surr,
                       active);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}

extern "C" int bm_da_accept(const bm_demcz* s, const double* chi2, const int32_t* flags, const double* chi2_surr,
                            const int32_t* active, void* stream) {
    int st = check_demcz(s);
    if (st != BM_OK) return st;
    if (!chi2 || !chi2_surr || !active || !s->lp_surr) return BM_EINVAL;
    hipLaunchKernelGGL(k_demcz_accept, dim3(1), dim3(1024), 0, (hipStream_t)stream, *s, chi2, flags, chi2_surr, active,
                       1);
    BM_CHECK_HIP(hipGetLastError());
    return BM_OK;
}
