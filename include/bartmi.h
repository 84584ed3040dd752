/*
 * bartmi.h -- C ABI of the MI355X transmission forward model.
 *
 * The library computes the transmission spectrum of an exoplanet atmosphere the way
 * the BART forward model does inside its MCMC loop (Harrington et al., "BART I",
 * arXiv:2104.12522): an atmosphere (temperature and composition per layer, Sec. 3)
 * is turned into extinction by interpolating pre-computed per-molecule opacity
 * tables in temperature (Sec. 3, Sec. 4 items 3-4), optical depth is integrated
 * along slant chords through spherical layers and the absorbed fraction of each
 * annulus (2 pi r) is integrated over altitude (Sec. 6.1), and the spectrum is
 * binned over channels and compared with data by chi^2 (Sec. 3). The opacity tables
 * themselves are built line by line with Voigt profiles (Sec. 4, Sec. 6.1.1).
 *
 * Conventions for every call
 *  - Array arguments are DEVICE pointers unless the comment says "host". The caller
 *    owns every buffer; the library never frees, retains or reallocates them.
 *  - Every call is asynchronous on the HIP stream passed as `stream` (a hipStream_t,
 *    NULL = the default stream). Argument and shape errors are detected before any
 *    work is enqueued and returned synchronously; nothing is enqueued then.
 *  - Arrays are row-major, wavenumber fastest. Layer index 0 is the deepest layer
 *    (highest pressure); radii increase with the layer index.
 *  - Units are CGS: cm, K, cm^-1 for wavenumbers, cm^2/molecule for cross sections,
 *    cm^5/molecule^2 for collision-induced absorption, cm^-1 for extinction; pressures
 *    in bar.
 *  - `dtype` (BM_F32 or BM_F64) is the element type of opacity tables, extinction and
 *    optical depth (CIA tables are always double). Transit depths, radii, temperatures and densities are always
 *    double. Geometry (radii, chord lengths) is computed in double; in BM_F32 mode the
 *    chord weights are rounded once to float and the impact-parameter integral is
 *    accumulated in double.
 *  - Physical problems of one sample never fail a call: they set bits of that sample's
 *    int32 flag word (BM_FLAG_*). A sample with BM_FLAG_RADIUS gets NaN depths.
 *  - Calls on different streams may run concurrently as long as they do not share
 *    output buffers or a workspace.
 */
#ifndef BARTMI_H
#define BARTMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes (return values) ---------------------------------------------- */
#define BM_OK 0
#define BM_EINVAL -1       /* NULL pointer or invalid scalar argument */
#define BM_ESHAPE -2       /* sizes inconsistent or outside the supported range */
#define BM_EHIP -3         /* the HIP runtime reported an error when enqueuing */
#define BM_ENOSPACE -4     /* the caller's workspace is smaller than required */

/* ---- element types --------------------------------------------------------------- */
#define BM_F32 0
#define BM_F64 1

/* ---- per-sample flag bits ---------------------------------------------------------- */
#define BM_FLAG_T_CLAMP 1     /* a layer temperature lay outside a table's T range (clamped) */
#define BM_FLAG_SUM_X 2       /* absorber mixing ratios sum to >= 1 (filler set to zero)    */
#define BM_FLAG_RADIUS 4      /* hydrostatic radius invalid (1/r <= 0): depths are NaN       */
#define BM_FLAG_NONFINITE 8   /* a parameter or a layer temperature is not finite or <= 0   */

/* ---- temperature-profile modes ------------------------------------------------------ */
#define BM_TP_ISOTHERMAL 0    /* params: [T, log10 x_1..x_S, R_ref/R_J]                      */
#define BM_TP_LINE2013 1      /* params: [log10 kappa, log10 g1, log10 g2, alpha, beta,
                                          log10 x_1..x_S, R_ref/R_J]  (Sec. 6.3, Sec. 7:
                                          five-parameter profile of Line et al. 2013)        */

#define BM_MAX_SPECIES 8
#define BM_MAX_LAYERS 256
#define BM_MAX_TEMPS 64

/* Returns a static string for a status code (never freed). */
const char* bm_status_string(int status);

/* Library ABI version (major * 100 + minor). */
int bm_version(void);

/* Fixed constants of a transmission model (host values, copied by every call).
 * Sec. 6.2 and Sec. 7: a hot Jupiter resembling HD 189733 b; the radius parameter
 * applies at p_ref; filler gas H2:He in the ratio h2_frac : 1 - h2_frac. */
typedef struct bm_planet {
    double rs_cm;       /* stellar radius: depth = (projected opaque area) / (pi rs^2)     */
    double tstar;       /* stellar temperature, K (T(p) irradiation)                        */
    double rstar_cm;    /* stellar radius used by the T(p) irradiation temperature          */
    double a_cm;        /* orbital semi-major axis                                           */
    double tint;        /* internal temperature of the T(p) profile, K                       */
    double g_nom;       /* surface gravity at r_nom, cm s^-2; GM = g_nom r_nom^2             */
    double r_nom_cm;    /* nominal radius defining the planet mass                           */
    double p_ref_bar;   /* pressure at which the radius parameter R_ref applies              */
    double h2_frac;     /* H2 share of the filler gas (0.85)                                  */
    double m_h2_amu;    /* H2 mass                                                            */
    double m_he_amu;    /* He mass                                                            */
} bm_planet;

/* A forward-model instance: tables, grids, observation and constants. Pointers are
 * borrowed. One call may mix up to 4 distinct models (all of one dtype). */
typedef struct bm_model {
    int32_t dtype;        /* BM_F32 or BM_F64: element type of sigma                        */
    int32_t n_species;    /* S, 1..BM_MAX_SPECIES                                          */
    int32_t n_temp;       /* NT, 2..BM_MAX_TEMPS, temperatures of the opacity tables       */
    int32_t n_layers;     /* L, 2..BM_MAX_LAYERS                                           */
    int32_t n_nu;         /* Nnu >= 1, output wavenumbers                                  */
    int32_t n_temp_cia;   /* NTc: 0 = no CIA, else 2..BM_MAX_TEMPS                         */
    int32_t tp_mode;      /* BM_TP_ISOTHERMAL or BM_TP_LINE2013                             */
    int32_t bin_width;    /* channel width in wavenumber points for binning; 0 = none      */
    const void* sigma;    /* device [S][NT][L][Nnu] cross sections on the layer pressures  */
    const double* temp;   /* device [NT], strictly increasing                               */
    const double* cia;    /* device [NTc][Nnu] H2-H2 CIA coefficient, or NULL. Always double:
                             values ~1e-45 cm^5/molecule^2 are not representable in float */
    const double* temp_cia; /* device [NTc], strictly increasing, or NULL                   */
    const double* p_bar;  /* device [L], layer pressures, strictly decreasing               */
    const double* data;   /* device [Nnu/bin_width] observed channel depths, or NULL        */
    const double* err;    /* device [Nnu/bin_width] their 1-sigma errors, or NULL           */
    double mass_amu[BM_MAX_SPECIES]; /* host values: absorber masses                        */
    bm_planet planet;
} bm_model;

/* Number of parameters of a sample: (1 or 5) + S + 1. */
int bm_n_params(const bm_model* model);

/* ---- a1-a2: atmosphere -------------------------------------------------------------
 * Sec. 3 (profile generator: T(p) and constant-with-height abundances per layer) and
 * Sec. 6.2 (radius given at the reference pressure). For each of B samples with
 * parameters params[b][0..P) (row stride `param_stride` >= P), writes
 * temp[b][L] (K), n_species[b][S][L] and n_h2[b][L] (molecules cm^-3), radius[b][L]
 * (cm, hydrostatic with g = GM/r^2) and flags[b]. All outputs double, device. */
int bm_atmosphere(const bm_model* model, const double* params, int param_stride, int B,
                  double* temp, double* n_species, double* n_h2, double* radius,
                  int32_t* flags, void* stream);

/* ---- a3: extinction ------------------------------------------------------------------
 * Sec. 3 and Sec. 6.1.1 (the RT interpolates the opacity table to each layer's
 * temperature; the table lives on the layer pressures):
 *   ext[l][k] = sum_i n_species[i][l] sigma_i(T_l)[l][k] + n_h2[l]^2 cia(T_l)[k],
 * linear interpolation in T, clamped (BM_FLAG_T_CLAMP ORed into *flags).
 * temp [L], n_species [S][L], n_h2 [L] (ignored without CIA) are device doubles;
 * ext is device [L][Nnu] of model->dtype; flags is a device int32 (ORed, not cleared). */
int bm_extinction(const bm_model* model, const double* temp, const double* n_species,
                  const double* n_h2, void* ext, int32_t* flags, void* stream);

/* ---- a4: chord optical depth ---------------------------------------------------------
 * Sec. 6.1 (slant path lengths through the layers at several altitudes): impact
 * parameters b_j = radius[j]; trapezoid in path length along both chord halves,
 *   tau[j][k] = sum_{l=j}^{L-2} (s_{j,l+1} - s_{j,l}) (ext[l][k] + ext[l+1][k]),
 *   s_{j,l} = sqrt(r_l^2 - r_j^2),   tau[L-1][k] = 0.
 * radius [L] device double, strictly increasing; ext, tau device [L][Nnu] of dtype. */
int bm_optical_depth(const double* radius, const void* ext, int L, int n_nu, int dtype,
                     void* tau, void* stream);

/* ---- a5: transit depth -----------------------------------------------------------------
 * Sec. 6.1 (transmission times 2 pi r integrated over altitude): opaque disk inside
 * radius[0], trapezoid in impact parameter, accumulated in double:
 *   depth[k] = [r_0^2 + sum_{j=0}^{L-2} (r_{j+1}-r_j)(f_j r_j + f_{j+1} r_{j+1})] / rs^2,
 *   f_j = 1 - exp(-tau[j][k]).
 * radius [L], depth [Nnu] device doubles; tau device [L][Nnu] of dtype. */
int bm_transit_depth(const double* radius, const void* tau, int L, int n_nu, int dtype,
                     double rs_cm, double* depth, void* stream);

/* ---- a6: channel binning and chi^2 ----------------------------------------------------
 * Sec. 3 (the spectrum integrator produces per-channel predictions; MC3 computes chi^2)
 * and Sec. 6.3 (channels with perfect transmission over their ranges): binned[b][c] =
 * mean of depth[b][c*w .. c*w+w), c < Nnu / w (a ragged tail is dropped);
 * chi2[b] = sum_c ((binned[b][c] - data[c]) / err[c])^2 when data and err are not NULL.
 * depth [B][Nnu], binned [B][Nnu/w], data/err [Nnu/w], chi2 [B]: device doubles. */
int bm_bin_chi2(const double* depth, int B, int n_nu, int bin_width, const double* data,
                const double* err, double* binned, double* chi2, void* stream);

/* ---- a1-a6 fused: batched forward model ------------------------------------------------
 * Sec. 3 and Sec. 4 items 8-9 (long-lived forward-model workers sharing one copy of the
 * opacity table): B samples, sample b uses models[instance[b]] (instance is a HOST
 * array, NULL = all use models[0]); params device [B][param_stride].
 * Outputs, concatenated over samples in order: depth (device double, sample b at offset
 * sum_{b'<b} Nnu(b')), binned (device double, offset sum_{b'<b} Nnu(b')/w(b'); NULL to
 * skip; needs bin_width > 0 in every used model), chi2 (device double [B] against each
 * model's data/err; NULL to skip; needs binned and data/err in every used model), flags
 * (device int32 [B]).
 * `active` (device int32 [B], or NULL = all) skips samples whose entry is 0: their
 * depth, binned, chi2 and flags entries are left untouched (delayed acceptance runs the
 * exact model only for the proposals its first stage passed, with static shapes).
 * The workspace (device, `workspace_bytes` >= bm_workspace_size(...)) holds per-sample
 * records; it needs no initialisation. Calls sharing one workspace must be ordered on
 * one stream. Only kernels are enqueued (no memset or copy), so a call can be captured
 * in a HIP graph. */
size_t bm_workspace_size(const bm_model* models, int n_models, const int32_t* instance,
                         int B);
int bm_forward_batch(const bm_model* models, int n_models, const int32_t* instance,
                     const double* params, int param_stride, int B, const int32_t* active,
                     double* depth, double* binned, double* chi2, int32_t* flags,
                     void* workspace, size_t workspace_bytes, void* stream);

/* ---- DE-MCz sampler with delayed acceptance ----------------------------------------------
 * Sec. 3 and Sec. 5: MC3's differential-evolution samplers (DEMC, ter Braak 2006; the
 * archive-based DEMCzs, ter Braak & Vrugt 2008), here in archive form for a whole
 * generation of chains at once, so every chain's forward model of a generation is one
 * batched bm_forward_batch call. Proposal y = x + gamma (z_r1 - z_r2) + e from two
 * distinct archive rows, gamma = 2.38/sqrt(2d) (1 every 10th generation), e ~
 * N(0, (eps_scale width)^2); log posterior -chi^2/2 in the uniform prior box;
 * Metropolis acceptance. Delayed acceptance (Christen & Fox 2005): a surrogate chi^2
 * screens proposals (stage 1) and the exact model decides among the survivors with the
 * corrected ratio (stage 2), which keeps the exact posterior.
 * Random numbers: SplitMix64 outputs addressed by (generation, chain, slot) counters.
 * All pointers are device pointers owned by the caller; the sampler state lives in them,
 * including the generation and archive counters, so a generation can be graph-captured
 * and replayed. */
typedef struct bm_demcz {
    int32_t n_chains;   /* C, 1..1024                                                       */
    int32_t n_params;   /* d, 1..32                                                         */
    int32_t z_cap;      /* archive capacity in rows (>= 2)                                  */
    int32_t thin;       /* append the C chain states to the archive every `thin` generations */
    int32_t hist_cap;   /* generations the history buffer can hold (0 when history is NULL) */
    int32_t pad;
    uint64_t seed;      /* random stream                                                     */
    double eps_scale;   /* jitter sd as a fraction of each prior width (e.g. 1e-6)           */
    double* x;          /* [C][d] current states                                             */
    double* lp;         /* [C] log posterior of the current states                           */
    double* lp_surr;    /* [C] surrogate log posterior of the current states, or NULL        */
    double* prop;       /* [C][d] proposals written by bm_demcz_propose                      */
    double* z;          /* [z_cap][d] archive of past states                                 */
    int64_t* counters;  /* [2]: generation, archive rows in use                              */
    int64_t* n_accept;  /* [C][2]: stage-1 passes (delayed acceptance), acceptances          */
    double* history;    /* [hist_cap][C][d] states after each generation, or NULL            */
    const double* lo;   /* [d] prior box lower bounds                                        */
    const double* hi;   /* [d] prior box upper bounds                                        */
} bm_demcz;

/* Chains at uniform prior draws, archive with z_init further draws, counters reset. */
int bm_demcz_init(const bm_demcz* s, int z_init, void* stream);
/* Log posterior (and surrogate log posterior) of the current states from their chi^2
 * (device [C]; either may be NULL) and forward-model flags (device [C] or NULL). */
int bm_demcz_set_lp(const bm_demcz* s, const double* chi2, const int32_t* flags,
                    const double* chi2_surr, void* stream);
/* Proposals of the current generation into s->prop. */
int bm_demcz_propose(const bm_demcz* s, void* stream);
/* Metropolis acceptance of the proposals given their chi^2 [C] and flags [C] (or NULL);
 * records history, appends to the archive, advances the generation. */
int bm_demcz_accept(const bm_demcz* s, const double* chi2, const int32_t* flags, void* stream);
/* Delayed acceptance stage 1: active[c] = 1 when proposal c passes the surrogate test. */
int bm_da_screen(const bm_demcz* s, const double* chi2_surr, int32_t* active, void* stream);
/* Delayed acceptance stage 2 for the active proposals (exact chi^2 [C], flags [C] or
 * NULL, surrogate chi^2 [C]); bookkeeping as bm_demcz_accept. */
int bm_da_accept(const bm_demcz* s, const double* chi2, const int32_t* flags,
                 const double* chi2_surr, const int32_t* active, void* stream);

/* ---- opacity table build (secondary path) -----------------------------------------------
 * Sec. 3 and Sec. 4 (first pass: a per-molecule cross-section table on the output
 * wavenumber grid, at the layer pressures and over a temperature grid), Sec. 6.1.1
 * (Voigt profile from the Faddeeva function, Eqs. 4-11), Sec. 4 (point sampling at the
 * output wavenumbers). For every (T, p) cell and line:
 *   S(T) = S296 (296/T)^1.5 exp(-c2 E''/T)/exp(-c2 E''/296)
 *          (1 - exp(-c2 nu0/T))/(1 - exp(-c2 nu0/296)),
 *   sigma_D = nu0/c sqrt(k_B T / m),  gamma_L = gamma296 (p/1 atm) (296/T)^0.5,
 *   sigma[T][p][k] += S(T) V(nu_k - nu0; sigma_D, gamma_L) for |nu_k - nu0| <=
 *   cutoff_hwhm * HWHM_V (Olivero-Longbothum Voigt HWHM), nu_k = nu_start + k dnu.
 * Line arrays are device doubles [n_lines] (mass per line in amu) and MUST be sorted by
 * nu0 ascending (as line lists are distributed); unsorted input gives wrong tables.
 * temp [NT <= BM_MAX_TEMPS] and p_bar [NP <= BM_MAX_LAYERS] are HOST doubles; sigma_out
 * is device [NT][NP][Nnu] of dtype and every element is written once (no zero-fill
 * needed). Each element is a double sum over lines in line order, rounded once: the
 * result is deterministic. On its first call on a device the library allocates 256
 * bytes of device memory there, held until the process ends. */
int bm_opacity_table_build(const double* nu0, const double* s296, const double* gamma296,
                           const double* elow, const double* mass_amu, int64_t n_lines,
                           const double* temp, int n_temp, const double* p_bar, int n_p,
                           double nu_start, double dnu, int n_nu, double cutoff_hwhm,
                           int dtype, void* sigma_out, void* stream);

/* Voigt profile V(x; sigma, gamma) = Re w(z) / (sigma sqrt(2 pi)), z = (x + i gamma) /
 * (sigma sqrt 2) (Eqs. 4-11), evaluated with the library's Faddeeva routine in double.
 * x and out are device doubles [n]. */
int bm_voigt(const double* x, int64_t n, double sigma, double gamma, double* out,
             void* stream);

#ifdef __cplusplus
}
#endif
#endif /* BARTMI_H */
