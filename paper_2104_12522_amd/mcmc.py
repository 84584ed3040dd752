"""DE-MCz retrieval driver: the batched forward model inside a differential-evolution MCMC.

Every generation of C chains is: bm_demcz_propose (one kernel), one bm_forward_batch call
over all C proposals (atmosphere, extinction, optical depth, depth, channels, chi^2),
bm_demcz_accept (one kernel). With a surrogate, stage 1 of delayed acceptance screens the
proposals and the exact forward model runs only for the survivors (masked, so shapes stay
static). The sampler state lives on the GPU, so whole runs of generations can be captured
in a HIP graph and replayed with no host work per generation.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import (BmDemcz, Forward, _check, _ptr, _stream, lib)


class DEMCz:
    """GPU state of a DE-MCz sampler (see bm_demcz in bartmi.h)."""

    def __init__(self, n_chains: int, lo, hi, seed: int, thin: int = 10, z_cap: int | None = None,
                 hist_cap: int = 0, eps_scale: float = 1e-6, surrogate: bool = False,
                 device="cuda"):
        lo = np.asarray(lo, dtype=np.float64)
        hi = np.asarray(hi, dtype=np.float64)
        d = lo.size
        self.C, self.d = n_chains, d
        f64 = dict(dtype=torch.float64, device=device)
        self.x = torch.zeros(n_chains, d, **f64)
        self.lp = torch.zeros(n_chains, **f64)
        self.lp_surr = torch.zeros(n_chains, **f64) if surrogate else None
        self.prop = torch.zeros(n_chains, d, **f64)
        self.z_cap = z_cap if z_cap is not None else 10 * d + n_chains * 1000
        self.z = torch.zeros(self.z_cap, d, **f64)
        self.counters = torch.zeros(2, dtype=torch.int64, device=device)
        self.n_accept = torch.zeros(n_chains, 2, dtype=torch.int64, device=device)
        self.history = torch.zeros(hist_cap, n_chains, d, **f64) if hist_cap else None
        self.lo = torch.as_tensor(lo, **f64)
        self.hi = torch.as_tensor(hi, **f64)
        st = BmDemcz()
        st.n_chains, st.n_params, st.z_cap, st.thin = n_chains, d, self.z_cap, thin
        st.hist_cap = hist_cap
        st.seed = seed & 0xFFFFFFFFFFFFFFFF
        st.eps_scale = eps_scale
        for name in ("x", "lp", "lp_surr", "prop", "z", "counters", "n_accept", "history", "lo", "hi"):
            setattr(st, name, _ptr(getattr(self, name)))
        self.struct = st

    def _r(self, fn, *args, stream=None):
        _check(getattr(lib(), fn)(C.byref(self.struct), *args, _stream(stream)), fn)

    def init(self, z_init: int | None = None, stream=None):
        self._r("bm_demcz_init", z_init if z_init is not None else 10 * self.d, stream=stream)

    def set_lp(self, chi2=None, flags=None, chi2_surr=None, stream=None):
        self._r("bm_demcz_set_lp", _ptr(chi2), _ptr(flags), _ptr(chi2_surr), stream=stream)

    def propose(self, stream=None):
        self._r("bm_demcz_propose", stream=stream)

    def accept(self, chi2, flags=None, stream=None):
        self._r("bm_demcz_accept", _ptr(chi2), _ptr(flags), stream=stream)

    def da_screen(self, chi2_surr, active, stream=None):
        self._r("bm_da_screen", _ptr(chi2_surr), _ptr(active), stream=stream)

    def da_accept(self, chi2, flags, chi2_surr, active, stream=None):
        self._r("bm_da_accept", _ptr(chi2), _ptr(flags), _ptr(chi2_surr), _ptr(active), stream=stream)

    @property
    def generation(self) -> int:
        return int(self.counters[0])

    @property
    def archive_size(self) -> int:
        return int(self.counters[1])


class Retrieval:
    """A DE-MCz retrieval of one model's observation (model.data / model.err set).

    ``surrogate`` (optional) maps a [C][d] parameter tensor to a [C] surrogate chi^2 on
    the same stream; it enables two-stage delayed acceptance."""

    def __init__(self, model, n_chains: int, lo, hi, seed: int, thin: int = 10,
                 hist_cap: int = 0, surrogate=None, eps_scale: float = 1e-6, z_cap=None):
        self.model = model
        self.fwd = Forward(model, n_chains, binned=True, chi2=True)
        self.s = DEMCz(n_chains, lo, hi, seed, thin=thin, hist_cap=hist_cap, z_cap=z_cap,
                       eps_scale=eps_scale, surrogate=surrogate is not None)
        self.surrogate = surrogate
        self.active = torch.ones(n_chains, dtype=torch.int32, device=self.s.x.device)

    def start(self, z_init: int | None = None):
        self.s.init(z_init)
        self.fwd(self.s.x)
        chi2_s = self.surrogate(self.s.x) if self.surrogate is not None else None
        self.s.set_lp(self.fwd.chi2, self.fwd.flags, chi2_s)

    def generation(self):
        s = self.s
        s.propose()
        if self.surrogate is None:
            self.fwd(s.prop)
            s.accept(self.fwd.chi2, self.fwd.flags)
        else:
            chi2_s = self.surrogate(s.prop)
            s.da_screen(chi2_s, self.active)
            self.fwd(s.prop, active=self.active)
            s.da_accept(self.fwd.chi2, self.fwd.flags, chi2_s, self.active)

    def run(self, n_gen: int):
        for _ in range(n_gen):
            self.generation()

    def capture(self, n_gen: int) -> torch.cuda.CUDAGraph:
        """A HIP graph of n_gen generations (replay it to advance the chains)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                self.run(n_gen)
        torch.cuda.current_stream().wait_stream(side)
        return g
