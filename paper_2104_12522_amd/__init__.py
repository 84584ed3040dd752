"""Python binding of libbartmi, the MI355X transmission forward model.

Argument marshalling only: every step of the forward model, the opacity build and the
surrogate runs in the library's HIP kernels. PyTorch provides device memory and
streams. The library must be built (``python -m paper_2104_12522_amd.build``); there
is no fallback: importing works without it, but every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

from . import _abi
from ._abi import (BM_OK, BM_F32, BM_F64, BM_FLAG_T_CLAMP, BM_FLAG_SUM_X, BM_FLAG_RADIUS,
                   BM_FLAG_NONFINITE, BM_TP_ISOTHERMAL, BM_TP_LINE2013, BM_MAX_SPECIES,
                   BmPlanet, BmModel, BmDemcz)

__all__ = [
    "lib", "Model", "atmosphere", "extinction", "optical_depth", "transit_depth", "bin_chi2",
    "forward_batch", "Forward", "opacity_table_build", "voigt", "BM_F32", "BM_F64",
    "BM_FLAG_T_CLAMP", "BM_FLAG_SUM_X", "BM_FLAG_RADIUS", "BM_FLAG_NONFINITE",
    "BM_TP_ISOTHERMAL", "BM_TP_LINE2013",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbartmi.so")


class BartmiError(RuntimeError):
    pass


def lib() -> C.CDLL:
    return _abi.load(LIB_PATH)


def _check(status: int, what: str) -> None:
    if status != BM_OK:
        msg = lib().bm_status_string(status).decode()
        raise BartmiError(f"{what}: {msg} ({status})")


def _stream(stream=None) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None) -> C.c_void_p:
    if t is None:
        return C.c_void_p(None)
    if not t.is_cuda:
        raise BartmiError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise BartmiError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _keep_for_stream(tensors, stream=None) -> None:
    """Temporaries a call reads on a stream other than the current one: the caching
    allocator must not hand their memory out again until that stream's work is done."""
    if stream is None or stream == torch.cuda.current_stream():
        return
    for t in tensors:
        if t is not None and t.is_cuda:
            t.record_stream(stream)


def _dtype_code(dt: torch.dtype) -> int:
    if dt == torch.float32:
        return BM_F32
    if dt == torch.float64:
        return BM_F64
    raise BartmiError(f"unsupported dtype {dt}")


def _dev(x, dtype=torch.float64, device="cuda") -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=device)


def planet_struct(planet) -> BmPlanet:
    """A bm_planet from any object with the planet attributes (see workloads.Planet)."""
    return BmPlanet(planet.rs_cm, planet.tstar, planet.rstar_cm, planet.a_cm, planet.tint,
                    planet.g_nom, planet.r_nom_cm, planet.p_ref_bar, planet.h2_frac,
                    planet.m_h2_amu, planet.m_he_amu)


class Model:
    """A forward-model instance: device tables and grids plus the bm_model struct that
    borrows them. Keeps the tensors alive as long as the model is."""

    def __init__(self, sigma: torch.Tensor, temps, p_bar, mass_amu, tp_mode: int, planet,
                 cia: torch.Tensor | None = None, cia_temps=None, bin_width: int = 0,
                 data=None, err=None, device="cuda", tau_max: float = 0.0,
                 nu_start: float = 0.0, dnu: float = 0.0, rayleigh: bool = False,
                 cloud: bool = False, cia_he: torch.Tensor | None = None, geometry: str = "transit",
                 tiles: bool = True):
        """cia_he: an H2-He CIA table on the CIA temperature grid; it is folded into the
        H2-H2 table once here (bm_cia_combine), since n_He / n_H2 is fixed by the filler
        split. tiles: also keep a tile-major copy of the tables (bm_sigma_tiles, the table's
        size) for the tile width of binned calls,
        floor(64 / bin_width) bin_width (64 without channels); the fused kernel reads it
        for calls with that tile width (transit geometry)."""
        if sigma.dim() != 4:
            raise BartmiError("sigma must be [S][NT][L][Nnu]")
        self.sigma = sigma.to(device).contiguous()
        self.dtype = self.sigma.dtype
        S, NT, L, NNU = self.sigma.shape
        self.temps = _dev(temps, device=device)
        self.p_bar = _dev(p_bar, device=device)
        # CIA coefficients (~1e-45 cm^5/molecule^2) are kept in double whatever the dtype
        self.cia = None if cia is None else _dev(cia, device=device)
        if cia_he is not None:
            if self.cia is None:
                raise BartmiError("an H2-He CIA table needs the H2-H2 table and its temperature grid")
            he = _dev(cia_he, device=device)
            if tuple(he.shape) != tuple(self.cia.shape):
                raise BartmiError("the CIA tables must share the temperature and wavenumber grids")
            h = float(planet.h2_frac)
            combined = torch.empty_like(self.cia)
            _check(lib().bm_cia_combine(_ptr(self.cia), _ptr(he), (1.0 - h) / h if h > 0 else 0.0,
                                        self.cia.numel(), _ptr(combined), _stream(None)), "bm_cia_combine")
            self.cia = combined
        self.cia_temps = None if cia_temps is None else _dev(cia_temps, device=device)
        self.data = None if data is None else _dev(data, device=device)
        self.err = None if err is None else _dev(err, device=device)
        self.planet = planet
        st = BmModel()
        st.dtype = _dtype_code(self.dtype)
        st.n_species, st.n_temp, st.n_layers, st.n_nu = S, NT, L, NNU
        st.n_temp_cia = 0 if self.cia is None else self.cia.shape[0]
        st.tp_mode = tp_mode
        st.bin_width = bin_width
        st.sigma = _ptr(self.sigma)
        st.temp = _ptr(self.temps)
        st.cia = _ptr(self.cia)
        st.temp_cia = _ptr(self.cia_temps)
        st.p_bar = _ptr(self.p_bar)
        st.data = _ptr(self.data)
        st.err = _ptr(self.err)
        m = np.zeros(BM_MAX_SPECIES)
        m[:S] = np.asarray(mass_amu, dtype=np.float64)
        for i in range(BM_MAX_SPECIES):
            st.mass_amu[i] = float(m[i])
        st.planet = planet_struct(planet)
        st.tau_max = float(tau_max)
        if rayleigh and not dnu > 0:
            raise BartmiError("Rayleigh scattering needs the wavenumber grid (nu_start, dnu)")
        st.nu_start, st.dnu = float(nu_start), float(dnu)
        st.rayleigh, st.cloud = int(bool(rayleigh)), int(bool(cloud))
        if geometry not in ("transit", "eclipse"):
            raise BartmiError("geometry is 'transit' or 'eclipse'")
        st.geometry = 0 if geometry == "transit" else 1
        self.geometry = geometry
        self.struct = st
        self.sigma_tiles = None
        tw = (64 // bin_width) * bin_width if 1 <= bin_width <= 64 else 64
        # transit only (the emission kernel reads sigma); a model the library rejects gets no
        # copy here, and its calls report the error
        if tiles and geometry == "transit" and lib().bm_sigma_tiles_bytes(C.byref(st), tw) > 0:
            self.build_tiles(tw)

    def build_tiles(self, tile_w: int):
        """(Re)builds the tile-major table copy for tile width tile_w (bm_sigma_tiles)."""
        st = self.struct
        st.sigma_tiles, st.tile_w = None, 0
        self.sigma_tiles = None
        n = lib().bm_sigma_tiles_bytes(C.byref(st), int(tile_w))
        if n == 0:
            raise BartmiError(f"bm_sigma_tiles_bytes: invalid model or tile width {tile_w}")
        self.sigma_tiles = torch.empty(n // self.sigma.element_size(), dtype=self.dtype, device=self.sigma.device)
        _check(lib().bm_sigma_tiles(C.byref(st), int(tile_w), _ptr(self.sigma_tiles), n, _stream(None)),
               "bm_sigma_tiles")
        st.sigma_tiles, st.tile_w = _ptr(self.sigma_tiles), int(tile_w)

    @property
    def n_species(self):
        return self.struct.n_species

    @property
    def n_layers(self):
        return self.struct.n_layers

    @property
    def n_nu(self):
        return self.struct.n_nu

    @property
    def n_params(self) -> int:
        return lib().bm_n_params(C.byref(self.struct))

    @property
    def n_bins(self) -> int:
        w = self.struct.bin_width
        return self.n_nu // w if w > 0 else 0

    def set_observation(self, data, err):
        self.data = _dev(data, device=self.sigma.device)
        self.err = _dev(err, device=self.sigma.device)
        self.struct.data = _ptr(self.data)
        self.struct.err = _ptr(self.err)


# ------------------------------------------------------------------------------- steps
def atmosphere(model: Model, params: torch.Tensor, stream=None):
    """Steps a1-a2 for B samples: returns temp [B][L], n_species [B][S][L], n_h2 [B][L],
    radius [B][L] (double) and flags [B] (int32)."""
    params = _dev(params, device=model.sigma.device)
    if params.dim() == 1:
        params = params[None]
    B, P = params.shape
    L, S = model.n_layers, model.n_species
    dev = params.device
    temp = torch.empty(B, L, dtype=torch.float64, device=dev)
    nsp = torch.empty(B, S, L, dtype=torch.float64, device=dev)
    nh2 = torch.empty(B, L, dtype=torch.float64, device=dev)
    rad = torch.empty(B, L, dtype=torch.float64, device=dev)
    flags = torch.empty(B, dtype=torch.int32, device=dev)
    _check(lib().bm_atmosphere(C.byref(model.struct), _ptr(params), P, B, _ptr(temp), _ptr(nsp),
                               _ptr(nh2), _ptr(rad), _ptr(flags), _stream(stream)), "bm_atmosphere")
    return dict(temp=temp, n_species=nsp, n_h2=nh2, radius=rad, flags=flags)


def extinction(model: Model, temp, n_species, n_h2=None, stream=None):
    """Step a3 for one atmosphere: ext [L][Nnu] in the model dtype, flags (int32 [1])."""
    dev = model.sigma.device
    temp = _dev(temp, device=dev)
    n_species = _dev(n_species, device=dev)
    n_h2 = None if n_h2 is None else _dev(n_h2, device=dev)
    ext = torch.empty(model.n_layers, model.n_nu, dtype=model.dtype, device=dev)
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    _check(lib().bm_extinction(C.byref(model.struct), _ptr(temp), _ptr(n_species), _ptr(n_h2),
                               _ptr(ext), _ptr(flags), _stream(stream)), "bm_extinction")
    return ext, flags


def optical_depth(radius, ext: torch.Tensor, stream=None) -> torch.Tensor:
    """Step a4: tau [L][Nnu] from radii [L] and extinction [L][Nnu]."""
    radius = _dev(radius, device=ext.device)
    ext = ext.contiguous()
    L, N = ext.shape
    tau = torch.empty_like(ext)
    _check(lib().bm_optical_depth(_ptr(radius), _ptr(ext), L, N, _dtype_code(ext.dtype), _ptr(tau),
                                  _stream(stream)), "bm_optical_depth")
    return tau


def transit_depth(radius, tau: torch.Tensor, rs_cm: float, stream=None) -> torch.Tensor:
    """Step a5: depth [Nnu] (double)."""
    radius = _dev(radius, device=tau.device)
    tau = tau.contiguous()
    L, N = tau.shape
    depth = torch.empty(N, dtype=torch.float64, device=tau.device)
    _check(lib().bm_transit_depth(_ptr(radius), _ptr(tau), L, N, _dtype_code(tau.dtype),
                                  C.c_double(rs_cm), _ptr(depth), _stream(stream)), "bm_transit_depth")
    return depth


def bin_chi2(depth: torch.Tensor, bin_width: int, data=None, err=None, stream=None):
    """Step a6: binned [B][Nnu/w] and chi2 [B] (None without data)."""
    if depth.dim() == 1:
        depth = depth[None]
    depth = depth.contiguous()
    B, N = depth.shape
    nb = N // bin_width
    binned = torch.empty(B, nb, dtype=torch.float64, device=depth.device)
    chi2 = None
    if data is not None:
        data = _dev(data, device=depth.device)
        err = _dev(err, device=depth.device)
        chi2 = torch.empty(B, dtype=torch.float64, device=depth.device)
    _check(lib().bm_bin_chi2(_ptr(depth), B, N, bin_width, _ptr(data), _ptr(err), _ptr(binned),
                             _ptr(chi2), _stream(stream)), "bm_bin_chi2")
    return binned, chi2


# ------------------------------------------------------------------------------- fused
class Forward:
    """Reusable fused forward model (steps a1-a6) for a fixed batch layout: owns the
    workspace and output buffers so repeated calls allocate nothing."""

    def __init__(self, models, batch: int, instance=None, binned: bool = False,
                 chi2: bool = False, device="cuda"):
        self.models = list(models) if isinstance(models, (list, tuple)) else [models]
        n = len(self.models)
        self._structs = (BmModel * n)(*[m.struct for m in self.models])
        self.B = batch
        if instance is None:
            self._inst = None
            inst = [0] * batch
        else:
            inst = [int(i) for i in instance]
            if len(inst) != batch:
                raise BartmiError("instance must have one entry per sample")
            self._inst = (C.c_int32 * batch)(*inst)
        self.instance = inst
        self.n_nu = [self.models[i].n_nu for i in inst]
        self.n_bins = [self.models[i].n_bins for i in inst]
        self.depth_off = np.concatenate([[0], np.cumsum(self.n_nu)]).astype(np.int64)
        self.bin_off = np.concatenate([[0], np.cumsum(self.n_bins)]).astype(np.int64)
        ws = lib().bm_workspace_size(self._structs, n, self._inst, batch)
        if ws == 0 and batch > 0:
            raise BartmiError("bm_workspace_size rejected the models / batch")
        self.workspace = torch.zeros(max(int(ws), 256), dtype=torch.uint8, device=device)
        self.depth = torch.empty(int(self.depth_off[-1]), dtype=torch.float64, device=device)
        self.binned = (torch.empty(int(self.bin_off[-1]), dtype=torch.float64, device=device)
                       if (binned or chi2) else None)
        self.chi2 = torch.empty(batch, dtype=torch.float64, device=device) if chi2 else None
        self.flags = torch.empty(batch, dtype=torch.int32, device=device)
        self.param_stride = max(m.n_params for m in self.models)

    def __call__(self, params: torch.Tensor, stream=None, active: torch.Tensor | None = None):
        if params.shape[0] != self.B or params.dtype != torch.float64 or not params.is_contiguous():
            raise BartmiError("params must be a contiguous float64 [B][P] device tensor")
        if active is not None and (active.dtype != torch.int32 or active.numel() != self.B):
            raise BartmiError("active must be an int32 [B] device tensor")
        _check(lib().bm_forward_batch(self._structs, len(self.models), self._inst, _ptr(params),
                                      params.shape[1], self.B, _ptr(active), _ptr(self.depth),
                                      _ptr(self.binned), _ptr(self.chi2), _ptr(self.flags),
                                      _ptr(self.workspace), C.c_size_t(self.workspace.numel()),
                                      _stream(stream)),
               "bm_forward_batch")
        return self

    def call_noalloc(self, params: torch.Tensor, stream=None, active: torch.Tensor | None = None):
        """The same call through bm_forward_batch_noalloc: the library's fixed per-GPU array
        replaces this object's workspace (calls overlapping on one GPU race)."""
        if params.shape[0] != self.B or params.dtype != torch.float64 or not params.is_contiguous():
            raise BartmiError("params must be a contiguous float64 [B][P] device tensor")
        if active is not None and (active.dtype != torch.int32 or active.numel() != self.B):
            raise BartmiError("active must be an int32 [B] device tensor")
        _check(lib().bm_forward_batch_noalloc(self._structs, len(self.models), self._inst, _ptr(params),
                                              params.shape[1], self.B, _ptr(active), _ptr(self.depth),
                                              _ptr(self.binned), _ptr(self.chi2), _ptr(self.flags),
                                              _stream(stream)),
               "bm_forward_batch_noalloc")
        return self

    def tune(self, params: torch.Tensor, reps: int = 5, stream=None):
        """Autotune the fused kernel's launch configuration for this batch (bm_forward_tune);
        returns (chosen index, mean ms per call of every configuration). Overwrites the
        outputs; call before capturing the batch in a graph."""
        if params.shape[0] != self.B or params.dtype != torch.float64 or not params.is_contiguous():
            raise BartmiError("params must be a contiguous float64 [B][P] device tensor")
        n = lib().bm_forward_config_count()
        chosen = C.c_int(-1)
        times = (C.c_float * n)()
        _check(lib().bm_forward_tune(self._structs, len(self.models), self._inst, _ptr(params),
                                     params.shape[1], self.B, _ptr(self.depth), _ptr(self.binned),
                                     _ptr(self.chi2), _ptr(self.flags), _ptr(self.workspace),
                                     C.c_size_t(self.workspace.numel()), _stream(stream), reps,
                                     C.byref(chosen), times, n), "bm_forward_tune")
        return chosen.value, [float(t) for t in times]

    def set_config(self, config: int):
        """Pin a launch configuration for this batch (-1 returns to the default)."""
        _check(lib().bm_forward_set_config(self._structs, len(self.models), self._inst, self.B,
                                           config), "bm_forward_set_config")

    def spectrum(self, b: int) -> torch.Tensor:
        return self.depth[self.depth_off[b]:self.depth_off[b + 1]]

    def binned_spectrum(self, b: int) -> torch.Tensor:
        return self.binned[self.bin_off[b]:self.bin_off[b + 1]]


def forward_batch(models, params: torch.Tensor, instance=None, binned=False, chi2=False,
                  stream=None) -> Forward:
    params = _dev(params)
    if params.dim() == 1:
        params = params[None]
    f = Forward(models, params.shape[0], instance, binned=binned, chi2=chi2, device=params.device)
    return f(params, stream)


def forward_configs() -> list[str]:
    """Names of the fused kernel's launch configurations, by index."""
    return [lib().bm_forward_config_name(i).decode() for i in range(lib().bm_forward_config_count())]


class KernelTiming:
    """Context manager around bm_timing_start/stop: the fused kernel's launches inside the
    block are timed with HIP events on their streams. After the block, ``total_ms`` and
    ``launches`` hold the summed kernel time and the number of launches timed."""

    def __init__(self, capacity: int):
        self.capacity = capacity
        self.total_ms = 0.0
        self.launches = 0

    def __enter__(self):
        _check(lib().bm_timing_start(self.capacity), "bm_timing_start")
        return self

    def __exit__(self, *exc):
        tot = C.c_double(0.0)
        n = C.c_int64(0)
        _check(lib().bm_timing_stop(C.byref(tot), C.byref(n)), "bm_timing_stop")
        self.total_ms, self.launches = tot.value, n.value
        return False

    @property
    def mean_ms(self) -> float:
        return self.total_ms / self.launches if self.launches else float("nan")


# ------------------------------------------------------------------------------- opacity
def opacity_build_workspace(n_lines: int, device="cuda") -> torch.Tensor:
    """A device workspace for bm_opacity_table_build / bm_line_width_range."""
    nb = int(lib().bm_opacity_build_workspace(int(n_lines)))
    if nb == 0:
        raise BartmiError("invalid line count")
    return torch.empty(nb, dtype=torch.uint8, device=device)


def opacity_table_build(lines, temps, p_bar, nu_start: float, dnu: float, n_nu: int,
                        cutoff_hwhm: float = 25.0, dtype=torch.float32, device="cuda",
                        out: torch.Tensor | None = None, stream=None,
                        workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Cross-section table [NT][NP][Nnu] of one species. ``lines`` has attributes nu0,
    s296, gamma296, elow, mass_amu (numpy or torch, sorted by nu0). Builds that may run
    concurrently (other streams) need workspaces of their own."""
    arrs = [_dev(getattr(lines, f), device=device) for f in
            ("nu0", "s296", "gamma296", "elow", "mass_amu")]
    n = int(arrs[0].numel())
    temps = np.ascontiguousarray(np.asarray(temps, dtype=np.float64))
    p_bar = np.ascontiguousarray(np.asarray(p_bar, dtype=np.float64))
    if out is None:
        out = torch.empty(len(temps), len(p_bar), n_nu, dtype=dtype, device=device)
    if workspace is None:
        workspace = opacity_build_workspace(n, device=device)
    dp = C.POINTER(C.c_double)
    _check(lib().bm_opacity_table_build(*[_ptr(a) for a in arrs], n, temps.ctypes.data_as(dp),
                                        len(temps), p_bar.ctypes.data_as(dp), len(p_bar),
                                        C.c_double(nu_start), C.c_double(dnu), n_nu,
                                        C.c_double(cutoff_hwhm), _dtype_code(out.dtype),
                                        _ptr(out), _ptr(workspace), workspace.numel(),
                                        _stream(stream)), "bm_opacity_table_build")
    _keep_for_stream(arrs + [workspace], stream)
    return out


def line_width_range(lines, temps, p_bar, device="cuda", stream=None) -> np.ndarray:
    """(min sigma_D, max sigma_D, min gamma_L, max gamma_L) of the lines over the cells of
    these temperatures and pressures (bm_line_width_range); waits for the result."""
    arrs = [_dev(getattr(lines, f), device=device) for f in ("nu0", "gamma296", "mass_amu")]
    n = int(arrs[0].numel())
    temps = np.ascontiguousarray(np.asarray(temps, dtype=np.float64))
    p_bar = np.ascontiguousarray(np.asarray(p_bar, dtype=np.float64))
    ws = opacity_build_workspace(n, device=device)
    out = torch.empty(4, dtype=torch.float64, device=device)
    dp = C.POINTER(C.c_double)
    _check(lib().bm_line_width_range(*[_ptr(a) for a in arrs], n, temps.ctypes.data_as(dp), len(temps),
                                     p_bar.ctypes.data_as(dp), len(p_bar), _ptr(out), _ptr(ws), ws.numel(),
                                     _stream(stream)), "bm_line_width_range")
    return out.cpu().numpy()


class VoigtTable:
    """The paper's 3D table of Voigt profiles on the device (bm_voigt_table_build): nodes of
    Doppler and Lorentz widths (host arrays, strictly increasing), ``oversample`` fine
    samples per output interval ``dnu``, each profile reaching ``cutoff_hwhm`` Voigt HWHMs."""

    def __init__(self, sigma_nodes, gamma_nodes, dnu: float, oversample: int, cutoff_hwhm: float = 25.0,
                 device="cuda", stream=None):
        from ._abi import BmVoigtGrid
        self.sigma_nodes = np.ascontiguousarray(np.asarray(sigma_nodes, dtype=np.float64))
        self.gamma_nodes = np.ascontiguousarray(np.asarray(gamma_nodes, dtype=np.float64))
        g = BmVoigtGrid()
        g.n_sigma, g.n_gamma, g.oversample = self.sigma_nodes.size, self.gamma_nodes.size, int(oversample)
        g.sigma_nodes = self.sigma_nodes.ctypes.data
        g.gamma_nodes = self.gamma_nodes.ctypes.data
        g.dnu, g.cutoff_hwhm = float(dnu), float(cutoff_hwhm)
        self.grid = g
        self.bytes = int(lib().bm_voigt_table_bytes(C.byref(g)))
        if self.bytes == 0:
            raise BartmiError("invalid Voigt profile grid")
        self.table = torch.empty(self.bytes, dtype=torch.uint8, device=device)
        _check(lib().bm_voigt_table_build(C.byref(g), _ptr(self.table), self.bytes, _stream(stream)),
               "bm_voigt_table_build")

    @staticmethod
    def nodes_for(lines, temps, p_bar, n_sigma: int = 60, n_gamma: int = 60, margin: float = 1.01,
                  device="cuda"):
        """Log-spaced nodes over the Doppler and Lorentz widths the lines take in these
        cells (the range of expected widths, from bm_line_width_range), widened by `margin`
        at both ends."""
        s_lo, s_hi, g_lo, g_hi = line_width_range(lines, temps, p_bar, device=device)
        return (np.geomspace(s_lo / margin, s_hi * margin, n_sigma),
                np.geomspace(g_lo / margin, g_hi * margin, n_gamma))


def opacity_table_build_profiles(lines, temps, p_bar, nu_start: float, n_nu: int, table: VoigtTable,
                                 strength_cutoff: float = 0.0, dtype=torch.float32, device="cuda",
                                 out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Cross-section table [NT][NP][Nnu] in the paper's profile-table mode (Sec. 4 items 4-6):
    nearest tabulated profile, integer fine shift, strengths of lines sharing profile and
    shift summed, lines below strength_cutoff times the strongest ignored."""
    arrs = [_dev(getattr(lines, f), device=device) for f in
            ("nu0", "s296", "gamma296", "elow", "mass_amu")]
    n = int(arrs[0].numel())
    temps = np.ascontiguousarray(np.asarray(temps, dtype=np.float64))
    p_bar = np.ascontiguousarray(np.asarray(p_bar, dtype=np.float64))
    if out is None:
        out = torch.empty(len(temps), len(p_bar), n_nu, dtype=dtype, device=device)
    wsb = int(lib().bm_opacity_profiles_workspace(len(temps)))
    if wsb == 0:
        raise BartmiError("too many temperatures")
    ws = torch.empty(wsb, dtype=torch.uint8, device=device)
    dp = C.POINTER(C.c_double)
    _check(lib().bm_opacity_table_build_profiles(
        *[_ptr(a) for a in arrs], n, temps.ctypes.data_as(dp), len(temps), p_bar.ctypes.data_as(dp),
        len(p_bar), C.c_double(nu_start), n_nu, C.byref(table.grid), _ptr(table.table),
        C.c_double(strength_cutoff), _dtype_code(out.dtype), _ptr(out), _ptr(ws), wsb, _stream(stream)),
        "bm_opacity_table_build_profiles")
    _keep_for_stream(arrs + [ws], stream)
    return out


def voigt(x: torch.Tensor, sigma: float, gamma: float, stream=None) -> torch.Tensor:
    x = _dev(x)
    out = torch.empty_like(x)
    _check(lib().bm_voigt(_ptr(x), x.numel(), C.c_double(sigma), C.c_double(gamma), _ptr(out),
                          _stream(stream)), "bm_voigt")
    return out
