"""ctypes declarations mirroring include/bartmi.h."""
from __future__ import annotations

import ctypes as C
import os

BM_OK, BM_EINVAL, BM_ESHAPE, BM_EHIP, BM_ENOSPACE, BM_ESCRATCH = 0, -1, -2, -3, -4, -5
BM_NOALLOC_SCRATCH_BYTES = 64 << 20
BM_F32, BM_F64 = 0, 1
BM_FLAG_T_CLAMP, BM_FLAG_SUM_X, BM_FLAG_RADIUS, BM_FLAG_NONFINITE = 1, 2, 4, 8
BM_TP_ISOTHERMAL, BM_TP_LINE2013 = 0, 1
BM_MAX_SPECIES, BM_MAX_LAYERS, BM_MAX_TEMPS = 8, 256, 64
BM_MLP_MAX_LAYERS = 8
BM_GEMM_STORE, BM_GEMM_BIAS_SILU, BM_GEMM_BIAS, BM_GEMM_SILU_GRAD = 0, 1, 2, 3


class BmPlanet(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "rs_cm", "tstar", "rstar_cm", "a_cm", "tint", "g_nom", "r_nom_cm", "p_ref_bar",
        "h2_frac", "m_h2_amu", "m_he_amu")]


class BmModel(C.Structure):
    _fields_ = [
        ("dtype", C.c_int32), ("n_species", C.c_int32), ("n_temp", C.c_int32),
        ("n_layers", C.c_int32), ("n_nu", C.c_int32), ("n_temp_cia", C.c_int32),
        ("tp_mode", C.c_int32), ("bin_width", C.c_int32),
        ("sigma", C.c_void_p), ("temp", C.c_void_p), ("cia", C.c_void_p),
        ("temp_cia", C.c_void_p), ("p_bar", C.c_void_p), ("data", C.c_void_p),
        ("err", C.c_void_p),
        ("mass_amu", C.c_double * BM_MAX_SPECIES),
        ("planet", BmPlanet),
        ("tau_max", C.c_double), ("nu_start", C.c_double), ("dnu", C.c_double),
        ("rayleigh", C.c_int32), ("cloud", C.c_int32), ("geometry", C.c_int32), ("pad2", C.c_int32),
        ("sigma_tiles", C.c_void_p), ("tile_w", C.c_int32), ("pad3", C.c_int32),
    ]


class BmDemcz(C.Structure):
    _fields_ = [
        ("n_chains", C.c_int32), ("n_params", C.c_int32), ("z_cap", C.c_int32),
        ("thin", C.c_int32), ("hist_cap", C.c_int32), ("n_free", C.c_int32),
        ("seed", C.c_uint64), ("eps_scale", C.c_double),
        ("x", C.c_void_p), ("lp", C.c_void_p), ("lp_surr", C.c_void_p), ("prop", C.c_void_p),
        ("z", C.c_void_p), ("counters", C.c_void_p), ("n_accept", C.c_void_p),
        ("history", C.c_void_p), ("lo", C.c_void_p), ("hi", C.c_void_p),
        ("p_snooker", C.c_double), ("log_q", C.c_void_p), ("gamma_scale", C.c_double),
    ]


class BmVoigtGrid(C.Structure):
    _fields_ = [
        ("n_sigma", C.c_int32), ("n_gamma", C.c_int32), ("oversample", C.c_int32), ("pad", C.c_int32),
        ("sigma_nodes", C.c_void_p), ("gamma_nodes", C.c_void_p), ("dnu", C.c_double),
        ("cutoff_hwhm", C.c_double),
    ]


class BmMlp(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("max_batch", C.c_int32),
                ("dims", C.c_int32 * (BM_MLP_MAX_LAYERS + 1))] + [
        (n, C.c_void_p * BM_MLP_MAX_LAYERS)
        for n in ("w32", "w16", "b32", "gw", "gb", "mw", "vw", "mb", "vb", "z", "h")] + [
        ("dz", C.c_void_p * 2)]


_VP = C.c_void_p
_I = C.c_int
_D = C.c_double
_I64 = C.c_int64
_PM = C.POINTER(BmModel)

PROTOTYPES = {
    "bm_status_string": (C.c_char_p, [_I]),
    "bm_version": (_I, []),
    "bm_struct_size": (C.c_size_t, [_I]),
    "bm_cia_combine": (_I, [C.c_void_p, C.c_void_p, C.c_double, C.c_int64, C.c_void_p, C.c_void_p]),
    "bm_voigt_table_bytes": (C.c_size_t, [C.c_void_p]),
    "bm_voigt_table_build": (_I, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "bm_opacity_profiles_workspace": (C.c_size_t, [_I]),
    "bm_opacity_table_build_profiles": (_I, [C.c_void_p] * 5 + [C.c_int64, C.c_void_p, _I, C.c_void_p, _I,
                                             C.c_double, _I, C.c_void_p, C.c_void_p, C.c_double, _I,
                                             C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "bm_n_params": (_I, [_PM]),
    "bm_atmosphere": (_I, [_PM, _VP, _I, _I, _VP, _VP, _VP, _VP, _VP, _VP]),
    "bm_extinction": (_I, [_PM, _VP, _VP, _VP, _VP, _VP, _VP]),
    "bm_optical_depth": (_I, [_VP, _VP, _I, _I, _I, _VP, _VP]),
    "bm_transit_depth": (_I, [_VP, _VP, _I, _I, _I, _D, _VP, _VP]),
    "bm_bin_chi2": (_I, [_VP, _I, _I, _I, _VP, _VP, _VP, _VP, _VP]),
    "bm_workspace_size": (C.c_size_t, [_PM, _I, C.POINTER(C.c_int32), _I]),
    "bm_sigma_tiles_bytes": (C.c_size_t, [_PM, _I]),
    "bm_sigma_tiles": (_I, [_PM, _I, C.c_void_p, C.c_size_t, C.c_void_p]),
    "bm_forward_batch": (_I, [_PM, _I, C.POINTER(C.c_int32), _VP, _I, _I, _VP, _VP, _VP, _VP, _VP,
                              _VP, C.c_size_t, _VP]),
    "bm_forward_batch_noalloc": (_I, [_PM, _I, C.POINTER(C.c_int32), _VP, _I, _I, _VP, _VP, _VP, _VP, _VP,
                                      _VP]),
    "bm_forward_config_count": (_I, []),
    "bm_forward_config_name": (C.c_char_p, [_I]),
    "bm_forward_tune": (_I, [_PM, _I, C.POINTER(C.c_int32), _VP, _I, _I, _VP, _VP, _VP, _VP, _VP,
                             C.c_size_t, _VP, _I, C.POINTER(C.c_int), C.POINTER(C.c_float), _I]),
    "bm_forward_set_config": (_I, [_PM, _I, C.POINTER(C.c_int32), _I, _I]),
    "bm_timing_start": (_I, [_I]),
    "bm_timing_stop": (_I, [C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "bm_demcz_init": (_I, [C.POINTER(BmDemcz), _I, _VP]),
    "bm_demcz_set_lp": (_I, [C.POINTER(BmDemcz), _VP, _VP, _VP, _VP]),
    "bm_demcz_propose": (_I, [C.POINTER(BmDemcz), _VP]),
    "bm_demcz_accept": (_I, [C.POINTER(BmDemcz), _VP, _VP, _VP]),
    "bm_da_screen": (_I, [C.POINTER(BmDemcz), _VP, _VP, _VP]),
    "bm_da_accept": (_I, [C.POINTER(BmDemcz), _VP, _VP, _VP, _VP, _VP]),
    "bm_opacity_build_workspace": (C.c_size_t, [_I64]),
    "bm_opacity_table_build": (_I, [_VP, _VP, _VP, _VP, _VP, _I64, C.POINTER(C.c_double), _I,
                                    C.POINTER(C.c_double), _I, _D, _D, _I, _D, _I, _VP, _VP,
                                    C.c_size_t, _VP]),
    "bm_line_width_range": (_I, [_VP, _VP, _VP, _I64, C.POINTER(C.c_double), _I, C.POINTER(C.c_double), _I,
                                 _VP, _VP, C.c_size_t, _VP]),
    "bm_voigt": (_I, [_VP, _I64, _D, _D, _VP, _VP]),
    "bm_gemm_bf16": (_I, [_I, _I, _I, _VP, _I, _I, _VP, _I, _I, _I, _VP, _VP, _I, _VP, _I, _VP, _I,
                          C.c_float, _VP]),
    "bm_mlp_set_input": (_I, [C.POINTER(BmMlp), _VP, _I, _VP, _I, _I, _VP, _VP, _VP]),
    "bm_mlp_forward": (_I, [C.POINTER(BmMlp), _I, _VP, _VP]),
    "bm_mlp_loss_grad": (_I, [C.POINTER(BmMlp), _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "bm_mlp_backward": (_I, [C.POINTER(BmMlp), _I, _VP]),
    "bm_adam_step": (_I, [C.POINTER(BmMlp), C.c_float, C.c_float, C.c_float, C.c_float, _I, _VP]),
    "bm_mlp_sync_bf16": (_I, [C.POINTER(BmMlp), _VP]),
    "bm_surrogate_chi2": (_I, [_VP, _I, _I, _VP, _VP, _VP, _VP, _VP, _VP]),
}

_cache: dict[str, C.CDLL] = {}


def load(path: str) -> C.CDLL:
    if path in _cache:
        return _cache[path]
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_2104_12522_amd.build); there is no fallback")
    lib = C.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _cache[path] = lib
    return lib
