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
#define BM_ESCRATCH -5     /* a no-allocation call needs more than the library's fixed array */

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

/* sizeof of a structure of this header, for bindings to check their own layouts:
 * which = 0 bm_planet, 1 bm_model, 2 bm_demcz, 3 bm_mlp, 4 bm_voigt_grid; 0 for any other. */
size_t bm_struct_size(int which);

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
    double tau_max;       /* Sec. 4 item 7, the optical-depth limit: in bm_forward_batch every
                             chord at or below (deeper than) one whose optical depth reaches
                             tau_max counts as opaque, f = 1; <= 0 or infinite = no limit
                             (the optical depth grows monotonically with depth, so this is
                             f = 1 wherever tau >= tau_max)                                    */
    double nu_start;      /* wavenumber of table column 0 (cm^-1); used by Rayleigh scattering */
    double dnu;           /* wavenumber step of the tables (cm^-1)                           */
    int32_t rayleigh;     /* 1: add H2 Rayleigh scattering n_H2 sigma_R(nu) to the extinction
                             (Sec. 3; sigma_R of Dalgarno & Williams 1962)                     */
    int32_t cloud;        /* 1: gray cloud deck (Sec. 3; cloud-top pressure of Sec. 7): one more
                             parameter, log10(p_cloud / bar), after the radius; in
                             bm_forward_batch every chord whose impact-parameter layer has
                             p >= p_cloud is opaque                                            */
    int32_t geometry;     /* BM_GEOM_TRANSIT (transit depth) or BM_GEOM_ECLIPSE (emergent
                             intensity, below); eclipse takes no cloud deck and no tau_max     */
    int32_t pad2;
    const void* sigma_tiles; /* device, or NULL: tile-major copy of sigma written by
                             bm_sigma_tiles for this model and tile width tile_w; read by
                             bm_forward_batch's fused kernel in place of sigma wherever its
                             tile width equals tile_w (else sigma is read)                   */
    int32_t tile_w;       /* 1..64: the wavenumbers per tile of sigma_tiles (ignored if NULL) */
    int32_t pad3;
} bm_model;

/* Geometries of bm_forward_batch's spectrum (bm_model.geometry).
 * BM_GEOM_ECLIPSE (Sec. 3 and Sec. 4, transit's emission spectra; Sec. 6, the intensity
 * spectra of the eclipse-geometry tests): plane-parallel layers at the hydrostatic radii,
 * vertical optical depth from the top by the trapezoid in height,
 *   tau_{L-1} = 0, tau_l = tau_{l+1} + (r_{l+1} - r_l)(e_l + e_{l+1}) / 2,
 * and the intensity emerging along the normal with the Planck function as source, the
 * deepest layer radiating from below and the two layers' mean source between them:
 *   I = B(T_0) e^{-tau_0} + sum_l (B(T_l) + B(T_{l+1}))/2 (e^{-tau_{l+1}} - e^{-tau_l}),
 *   B(T) = 2 h c^2 nu^3 / (exp(c2 nu / T) - 1)   (erg s^-1 cm^-2 sr^-1 (cm^-1)^-1),
 * which needs the wavenumber grid (nu_start, dnu). The spectrum buffer then holds I. */
#define BM_GEOM_TRANSIT 0
#define BM_GEOM_ECLIPSE 1

/* Number of parameters of a sample: (1 or 5) + S + 1 (+ 1 with a cloud deck). */
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
 *   ext[l][k] = sum_i n_species[i][l] sigma_i(T_l)[l][k] + n_h2[l]^2 cia(T_l)[k]
 *             (+ n_h2[l] sigma_R(nu_k) with model->rayleigh),
 * linear interpolation in T, clamped (BM_FLAG_T_CLAMP ORed into *flags).
 * temp [L], n_species [S][L], n_h2 [L] (ignored without CIA and Rayleigh) are device doubles;
 * ext is device [L][Nnu] of model->dtype; flags is a device int32 (ORed, not cleared). */
int bm_extinction(const bm_model* model, const double* temp, const double* n_species,
                  const double* n_h2, void* ext, int32_t* flags, void* stream);

/* ---- a3 (model setup): H2-He collision-induced absorption ------------------------------
 * Sec. 3 (CIA opacity sources): with the filler gas split H2:He in a fixed ratio h : 1 - h,
 * n_He = ((1 - h) / h) n_H2 in every layer, so the H2-He term n_H2 n_He K_He joins the
 * H2-H2 term as one table:
 *   out[i] = k_h2h2[i] + ratio * k_h2he[i],   ratio = (1 - h) / h,
 * to be passed as bm_model.cia (both tables on the same temperature grid). Device
 * doubles of n elements; out may alias k_h2h2. Asynchronous on `stream`. */
int bm_cia_combine(const double* k_h2h2, const double* k_h2he, double ratio, int64_t n, double* out,
                   void* stream);

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
 * exact model only for the proposals its first stage passed, with static shapes). A
 * masked transit call of one model over more than 16 samples builds the list of
 * requested samples on the device and launches the record preparation and the fused
 * kernel over that list (the requested samples' workgroups first), so its cost follows the
 * number of requested samples.
 * The workspace (device, `workspace_bytes` >= bm_workspace_size(...)) holds per-sample
 * records and the list of requested samples; it needs no initialisation. Calls sharing
 * one workspace must be ordered on one stream. Only kernels are enqueued (no memset or copy), so a call can be captured
 * in a HIP graph. */
size_t bm_workspace_size(const bm_model* models, int n_models, const int32_t* instance,
                         int B);
/* Tile-major copy of a model's opacity tables (the same values as sigma, rearranged).
 * bm_forward_batch's fused kernel reads the tables in tiles of tile_w consecutive
 * wavenumbers; in the row-major [S][NT][L][Nnu] layout each (species, temperature, layer)
 * row piece of a tile is a separate short read, which the copy turns into one contiguous
 * block per tile:
 *   out[s][k][t][l][c] = sigma[s][k][l][min(t tile_w + c, Nnu - 1)],
 *   t < n_tiles = ceil(Nnu / tile_w), c < tile_w, element type model->dtype
 * (the size of sigma, plus the ragged tail's padding).
 * bm_sigma_tiles_bytes gives the size (0 on invalid arguments); bm_sigma_tiles writes
 * `out` (device, caller-owned, out_bytes >= that size) on `stream` from model->sigma.
 * Set model->sigma_tiles = out and model->tile_w = tile_w to use it; the fused kernel
 * takes it for a run whose tile width is tile_w: floor(64 / bin_width) bin_width when the
 * call bins with 1 <= bin_width <= 64, else 64. Errors: BM_EINVAL (tile_w outside 1..64,
 * or a bad model), BM_ENOSPACE (out_bytes too small). */
size_t bm_sigma_tiles_bytes(const bm_model* model, int tile_w);
int bm_sigma_tiles(const bm_model* model, int tile_w, void* out, size_t out_bytes, void* stream);
int bm_forward_batch(const bm_model* models, int n_models, const int32_t* instance,
                     const double* params, int param_stride, int B, const int32_t* active,
                     double* depth, double* binned, double* chi2, int32_t* flags,
                     void* workspace, size_t workspace_bytes, void* stream);

/* ---- a1-a6 fused, no allocation -------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): bm_forward_batch with its workspace in
 * a library-owned device array of BM_NOALLOC_SCRATCH_BYTES (64 MiB), one per GPU, present
 * from the library's load on that GPU until the process ends. Arguments, outputs, launch
 * configuration and results are those of bm_forward_batch (bit-identical), without the
 * workspace arguments. The call allocates nothing and enqueues only kernels; the array
 * needs no clearing between calls (every call writes what it reads). Returns BM_ESCRATCH,
 * before any device work, when bm_workspace_size(models, n_models, instance, B) exceeds
 * the array (about 1600 samples of 100 layers x 30000 wavenumbers). Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams, other threads)
 * race, so order them on one stream. */
#define BM_NOALLOC_SCRATCH_BYTES (64u << 20)
int bm_forward_batch_noalloc(const bm_model* models, int n_models, const int32_t* instance,
                             const double* params, int param_stride, int B, const int32_t* active,
                             double* depth, double* binned, double* chi2, int32_t* flags,
                             void* stream);

/* ---- launch configurations and the autotuner --------------------------------------------
 * The fused kernel of bm_forward_batch has several launch configurations (waves per
 * workgroup; non-temporal or cached table loads). bm_forward_tune runs every
 * configuration on this exact batch (same arguments as bm_forward_batch without
 * `active`; it overwrites the outputs): one warm-up call, then `reps` calls timed with
 * HIP events, and remembers the fastest for the batch signature (dtype, species count,
 * CIA, and each run of samples: layers, wavenumbers, temperatures, bin width, count).
 * Later bm_forward_batch calls with that signature use it; untuned batches use cached table
 * loads with chord weights staged in LDS up to 512 workgroups (a few spectra), streamed
 * from L2 above that.
 * It waits for its events (host-synchronous) and refuses a stream under graph capture
 * (BM_EINVAL): tune first, then capture. `chosen` (host, may be NULL) receives the chosen
 * index, times_ms (host [n_times], may be NULL) the mean time per call of each
 * configuration (-1 where it was not run: FP64 has configuration 0 only). */
int bm_forward_config_count(void);
const char* bm_forward_config_name(int config);   /* static string; NULL if out of range */
int bm_forward_tune(const bm_model* models, int n_models, const int32_t* instance,
                    const double* params, int param_stride, int B, double* depth,
                    double* binned, double* chi2, int32_t* flags, void* workspace,
                    size_t workspace_bytes, void* stream, int reps, int* chosen,
                    float* times_ms, int n_times);
/* Pin configuration `config` for the signature of this batch (as if the autotuner had
 * chosen it); config -1 forgets the signature's entry. FP64 batches always run
 * configuration 0. */
int bm_forward_set_config(const bm_model* models, int n_models, const int32_t* instance, int B,
                          int config);

/* ---- kernel timing (measurement) ----------------------------------------------------------
 * Between bm_timing_start(capacity) and bm_timing_stop, the first `capacity` launches of
 * the fused forward kernel issued by bm_forward_batch outside graph capture each carry a
 * pair of HIP timing events that the dispatch records at the kernel's start and end
 * (hipExtLaunchKernel). bm_timing_stop waits for them and returns the summed kernel time
 * (ms) and the number of launches timed. One
 * session per process at a time (BM_EINVAL otherwise); the library creates and destroys
 * the events. */
int bm_timing_start(int capacity);
int bm_timing_stop(double* total_ms, int64_t* launches);

/* ---- opacity table build, profile-table mode (secondary path) ----------------------------
 * Sec. 4 items 4-6 and the paragraph after them, Sec. 6.1.1 (a 60 x 60 grid of profiles in
 * the f04 broadening test): the paper's own procedure.
 * Profile table: profile (i, j) is V(t delta; sigma_i, gamma_j) for fine offsets
 * t = -T..T, delta = dnu / oversample (samples aligned to the output grid),
 * T = floor(cutoff_hwhm HWHM(sigma_i, gamma_j) / delta) with the Olivero-Longbothum HWHM,
 * stored in single precision.
 * Build: for every (T, p) cell, each line takes S(T) and its Doppler and Lorentz widths
 * (as in bm_opacity_table_build), the nodes nearest its widths in ratio (geometric
 * midpoints of neighbouring nodes decide), the shift s = rint((nu0 - nu_start) / delta),
 * and is ignored when S(T) < strength_cutoff max_lines S(T) (S does not depend on p);
 * runs of consecutive lines (in centre order) with the same profile and shift have their
 * strengths summed before their profile is added; a line adds S P(k oversample - s) at
 * the output points k with |k oversample - s| <= T, summed in double in line order.
 * Node arrays are HOST doubles, strictly increasing and positive. */
typedef struct bm_voigt_grid {
    int32_t n_sigma;            /* Doppler-width nodes, 1..256                                   */
    int32_t n_gamma;            /* Lorentz-width nodes, 1..256                                   */
    int32_t oversample;         /* fine samples per output interval, 1..65536                    */
    int32_t pad;
    const double* sigma_nodes;  /* host [n_sigma], cm^-1                                         */
    const double* gamma_nodes;  /* host [n_gamma], cm^-1                                         */
    double dnu;                 /* output grid spacing (cm^-1) the profiles align to             */
    double cutoff_hwhm;         /* profile half extent in Voigt HWHMs                            */
} bm_voigt_grid;

/* Bytes of the device profile table for this grid (header + profiles); 0 when the grid is
 * invalid or the table would exceed 1.6e12 bytes. */
size_t bm_voigt_table_bytes(const bm_voigt_grid* grid);
/* Fills a caller-allocated device table of at least bm_voigt_table_bytes(grid) bytes: the
 * header is copied synchronously (the call returns after that copy), the profile values
 * are computed asynchronously on `stream`. */
int bm_voigt_table_build(const bm_voigt_grid* grid, void* table, size_t table_bytes, void* stream);
/* Bytes of the device workspace bm_opacity_table_build_profiles needs (0 if n_temp is out
 * of range): per-temperature strongest lines and the widest-window inputs. */
size_t bm_opacity_profiles_workspace(int n_temp);
/* The table-mode cross sections. Line arrays as bm_opacity_table_build (device doubles,
 * sorted by nu0); temp [n_temp] and p_bar [n_p] host doubles; grid and table as built by
 * bm_voigt_table_build (the grid's dnu is the output spacing); strength_cutoff >= 0 (0
 * keeps every line); sigma_out device [n_temp][n_p][n_nu] of dtype, every element written
 * once; deterministic. */
int bm_opacity_table_build_profiles(const double* nu0, const double* s296, const double* gamma296,
                                    const double* elow, const double* mass_amu, int64_t n_lines,
                                    const double* temp, int n_temp, const double* p_bar, int n_p,
                                    double nu_start, int n_nu, const bm_voigt_grid* grid,
                                    const void* table, double strength_cutoff, int dtype,
                                    void* sigma_out, void* workspace, size_t workspace_bytes,
                                    void* stream);

/* ---- DE-MCz sampler with delayed acceptance ----------------------------------------------
 * Sec. 3 and Sec. 5: MC3's differential-evolution samplers (DEMC, ter Braak 2006; the
 * archive-based DEMCzs, ter Braak & Vrugt 2008), here in archive form for a whole
 * generation of chains at once, so every chain's forward model of a generation is one
 * batched bm_forward_batch call. DE move: y = x + gamma (z_r1 - z_r2) + e from two
 * distinct archive rows, gamma = 2.38/sqrt(2k) (1 every 10th generation), e ~
 * N(0, (eps_scale width)^2). Snooker move (with probability p_snooker): a third distinct
 * archive row z; z_r1 and z_r2 projected onto the line through x and z; y = x +
 * gamma_s (projection difference), gamma_s ~ U[1.2, 2.2); proposal factor
 * (|y - z| / |x - z|)^(k-1) (no move when x = z), k the number of free parameters (a
 * parameter with lo = hi is held fixed: every state and archive row holds its value, so
 * no move changes it, and the chains move in the space of the other k). Log posterior
 * -chi^2/2 in the uniform
 * prior box; Metropolis-Hastings acceptance. Delayed acceptance (Christen & Fox 2005): a
 * surrogate chi^2 screens proposals (stage 1, with the proposal factor) and the exact
 * model decides among the survivors with the corrected ratio (stage 2, in which the
 * proposal factor cancels), which keeps the exact posterior. d <= 28.
 * Random numbers: SplitMix64 outputs addressed by (generation, chain, slot) counters.
 * All pointers are device pointers owned by the caller; the sampler state lives in them,
 * including the generation and archive counters, so a generation can be graph-captured
 * and replayed. */
typedef struct bm_demcz {
    int32_t n_chains;   /* C, 1..1024                                                       */
    int32_t n_params;   /* d, 1..28                                                         */
    int32_t z_cap;      /* archive capacity in rows (>= 2)                                  */
    int32_t thin;       /* append the C chain states to the archive every `thin` generations */
    int32_t hist_cap;   /* generations the history buffer can hold (0 when history is NULL) */
    int32_t n_free;     /* k: parameters with hi > lo (the others fixed); 0 reads as d       */
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
    const double* lo;   /* [d] prior box lower bounds (lo = hi holds a parameter fixed)      */
    const double* hi;   /* [d] prior box upper bounds                                        */
    double p_snooker;   /* probability of a snooker move per chain and generation (DEMCzs,
                           ter Braak & Vrugt 2008; 0.1 there), 0 = archive DE moves only     */
    double* log_q;      /* [C] log proposal factor of each chain's current proposal (0 for DE
                           moves); required when p_snooker > 0, else may be NULL           */
    double gamma_scale; /* DE-move step factor: gamma = gamma_scale 2.38/sqrt(2k) (ter Braak's
                           value for Gaussian targets); 0 is read as 1. The every-10th-
                           generation gamma = 1 moves are not scaled                         */
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
 * result is deterministic. `workspace` (device, caller-owned, workspace_bytes >=
 * bm_opacity_build_workspace(n_lines), no initialisation needed) receives the line list's
 * extremes that bound every cell's widest window; builds that may overlap need workspaces
 * of their own (calls on one stream are ordered). The library allocates nothing. Errors:
 * BM_EINVAL (NULL pointers, non-positive dnu, cutoff, temperature or pressure, bad dtype),
 * BM_ESHAPE (counts out of range), BM_ENOSPACE (workspace too small). */
size_t bm_opacity_build_workspace(int64_t n_lines);
int bm_opacity_table_build(const double* nu0, const double* s296, const double* gamma296,
                           const double* elow, const double* mass_amu, int64_t n_lines,
                           const double* temp, int n_temp, const double* p_bar, int n_p,
                           double nu_start, double dnu, int n_nu, double cutoff_hwhm,
                           int dtype, void* sigma_out, void* workspace, size_t workspace_bytes,
                           void* stream);

/* Range of the line widths over a set of cells (Sec. 4: the profile table spans the
 * expected Doppler and Lorentz widths; Eq. 2 and Eq. 3 widths as in
 * bm_opacity_table_build): range_out (device double [4]) = {min sigma_D, max sigma_D,
 * min gamma_L, max gamma_L} over the n_lines >= 1 lines (device doubles nu0, gamma296,
 * mass_amu; any order) and every temperature in temp [n_temp] and pressure in p_bar [n_p]
 * (HOST doubles, bar): sigma_D = nu0/c sqrt(k_B T / m) is extreme at the extreme nu0/sqrt(m)
 * and T, gamma_L = gamma296 (p/1 atm)(296/T)^0.5 at the extreme gamma296, p and T.
 * workspace as bm_opacity_table_build's. Asynchronous on `stream`. */
int bm_line_width_range(const double* nu0, const double* gamma296, const double* mass_amu,
                        int64_t n_lines, const double* temp, int n_temp, const double* p_bar,
                        int n_p, double* range_out, void* workspace, size_t workspace_bytes,
                        void* stream);

/* Voigt profile V(x; sigma, gamma) = Re w(z) / (sigma sqrt(2 pi)), z = (x + i gamma) /
 * (sigma sqrt 2) (Eqs. 4-11), evaluated with the library's Faddeeva routine in double.
 * x and out are device doubles [n]. */
int bm_voigt(const double* x, int64_t n, double sigma, double gamma, double* out,
             void* stream);

/* ---- learned surrogate for delayed acceptance --------------------------------------------
 * Sec. 1 motivates machine-learning surrogates of the forward model and Sec. 5 asks for
 * faster retrievals; here a multilayer perceptron maps the retrieval parameters to the
 * (standardised) binned spectrum and only screens proposals (stage 1 of bm_da_screen), so
 * the exact model still decides and the posterior is unchanged. Dense layers run on the
 * matrix cores in BF16 with FP32 accumulation; master weights and Adam moments are FP32.
 * Layer i (0 <= i < n_layers): z_i = h_i W_i^T + b_i with W_i [dims[i+1]][dims[i]]
 * row-major; h_{i+1} = silu(z_i) = z_i / (1 + exp(-z_i)) for hidden layers; the last
 * layer is linear. BF16 values are raw 16-bit patterns (round to nearest even).
 * All pointers are device pointers owned by the caller. */
#define BM_MLP_MAX_LAYERS 8

/* epilogues of bm_gemm_bf16 */
#define BM_GEMM_STORE 0      /* out_f32 = beta out_f32 + A B                               */
#define BM_GEMM_BIAS_SILU 1  /* z = A B + bias -> out_f32 (if not NULL); silu(z) -> out_bf16 */
#define BM_GEMM_BIAS 2       /* out_f32 = A B + bias                                       */
#define BM_GEMM_SILU_GRAD 3  /* out_bf16 = (A B) * silu'(aux)                              */

typedef struct bm_mlp {
    int32_t n_layers;                  /* 1..BM_MLP_MAX_LAYERS                              */
    int32_t max_batch;                 /* rows the activation buffers hold                  */
    int32_t dims[BM_MLP_MAX_LAYERS + 1]; /* widths: dims[0] input .. dims[n_layers] output  */
    float* w32[BM_MLP_MAX_LAYERS];     /* [dims[i+1]][dims[i]] FP32 master weights           */
    void* w16[BM_MLP_MAX_LAYERS];      /* same shape, BF16 copy used by the kernels          */
    float* b32[BM_MLP_MAX_LAYERS];     /* [dims[i+1]] biases                                 */
    float* gw[BM_MLP_MAX_LAYERS];      /* weight gradients (written by bm_mlp_backward)      */
    float* gb[BM_MLP_MAX_LAYERS];      /* bias gradients                                     */
    float* mw[BM_MLP_MAX_LAYERS];      /* Adam first moments of the weights (start at 0)     */
    float* vw[BM_MLP_MAX_LAYERS];      /* Adam second moments of the weights (start at 0)    */
    float* mb[BM_MLP_MAX_LAYERS];      /* Adam moments of the biases (start at 0)            */
    float* vb[BM_MLP_MAX_LAYERS];
    float* z[BM_MLP_MAX_LAYERS];       /* [max_batch][dims[i+1]] hidden pre-activations
                                          (i < n_layers - 1; the last may be NULL)           */
    void* h[BM_MLP_MAX_LAYERS];        /* [max_batch][dims[i]] BF16 layer inputs, h[0] the
                                          network input                                      */
    void* dz[2];                       /* two BF16 [max_batch][max(dims[1..])] scratch rows
                                          for back-propagated gradients                      */
} bm_mlp;

/* C[M][N] = A B in BF16 with FP32 accumulation on the matrix cores, with an epilogue.
 * A(m, k) = A[m lda + k] (trans_a 0) or A[k lda + m] (trans_a 1); B(k, n) = B[n ldb + k]
 * (trans_b 0, i.e. B stored as [N][K] like a weight matrix) or B[k ldb + n] (trans_b 1).
 * bias [N] FP32; aux [M][ldaux] FP32; out_f32 [M][ldo]; out_bf16 [M][ldob]. */
int bm_gemm_bf16(int M, int N, int K, const void* A, int lda, int trans_a, const void* B,
                 int ldb, int trans_b, int mode, const float* bias, const float* aux,
                 int ldaux, float* out_f32, int ldo, void* out_bf16, int ldob, float beta,
                 void* stream);
/* Network input h[0][b][j] = bf16((theta_rj - lo_j) / (hi_j - lo_j)) for j < P, zero for
 * P <= j < dims[0], with r = rows[b] (device int32 [B], e.g. a shuffled minibatch) or r = b
 * when rows is NULL; params device [*][param_stride], lo/hi device [P] doubles. */
int bm_mlp_set_input(const bm_mlp* net, const double* params, int param_stride,
                     const int32_t* rows, int B, int P, const double* lo, const double* hi,
                     void* stream);
/* Forward pass of B <= max_batch rows from h[0]; out [B][dims[n_layers]] FP32. */
int bm_mlp_forward(const bm_mlp* net, int B, float* out, void* stream);
/* Mean-squared-error loss on standardised targets, sum_bn (out_bn - t_bn)^2 / (B N) with
 * t_bn = (target_rn - mean_n) / scale_n, r = rows[b] (or b when rows is NULL); target
 * device doubles [*][N] (e.g. binned spectra), mean/scale device doubles [N] or both NULL
 * (t = target). Per-row sums of squares into row_loss [B] (FP32) and the gradient wrt out
 * into dz[0] (BF16). */
int bm_mlp_loss_grad(const bm_mlp* net, int B, const float* out, const double* target,
                     const int32_t* rows, const double* mean, const double* scale,
                     float* row_loss, void* stream);
/* Back-propagation from dz[0] (left by bm_mlp_loss_grad) through the activations of the
 * last bm_mlp_forward; writes gw and gb of every layer. */
int bm_mlp_backward(const bm_mlp* net, int B, void* stream);
/* One Adam step (Kingma & Ba 2015) with bias correction for step >= 1; refreshes w16. */
int bm_adam_step(const bm_mlp* net, float lr, float beta1, float beta2, float eps, int step,
                 void* stream);
/* w16 = bf16(w32) for every layer (after the caller initialises w32). */
int bm_mlp_sync_bf16(const bm_mlp* net, void* stream);
/* Surrogate chi^2 [B] (double) of standardised outputs out [B][N]: prediction_n = mean_n +
 * scale_n out_bn, chi^2 = sum_n ((prediction_n - data_n) / err_n)^2 (device doubles [N]). */
int bm_surrogate_chi2(const float* out, int B, int N, const double* mean, const double* scale,
                      const double* data, const double* err, double* chi2, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* BARTMI_H */
