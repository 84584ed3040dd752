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

from . import (BartmiError, BmDemcz, BmModel, Forward, _check, _ptr, _stream, lib)


class DEMCz:
    """GPU state of a DE-MCz sampler with snooker moves at rate p_snooker (see bm_demcz in
    bartmi.h). A parameter with lo = hi is held fixed; the step factor and the snooker
    proposal factor then count the free parameters only."""

    def __init__(self, n_chains: int, lo, hi, seed: int, thin: int = 10, z_cap: int | None = None,
                 hist_cap: int = 0, eps_scale: float = 1e-6, surrogate: bool = False,
                 p_snooker: float = 0.0, gamma_scale: float = 1.0, device="cuda"):
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
        self.log_q = torch.zeros(n_chains, **f64)
        st = BmDemcz()
        st.n_chains, st.n_params, st.z_cap, st.thin = n_chains, d, self.z_cap, thin
        st.hist_cap = hist_cap
        # parameters with lo = hi are held fixed; gamma and the snooker factor use the rest
        st.n_free = int(np.sum(hi > lo))
        st.seed = seed & 0xFFFFFFFFFFFFFFFF
        st.eps_scale = eps_scale
        st.p_snooker = float(p_snooker)
        st.gamma_scale = float(gamma_scale)
        for name in ("x", "lp", "lp_surr", "prop", "z", "counters", "n_accept", "history", "lo", "hi",
                     "log_q"):
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

    def load_state(self, x: torch.Tensor, archive: torch.Tensor, generation: int = 0):
        """Chain states and archive from elsewhere (e.g. a burn-in run); the log posteriors
        must be set again (set_lp) before the next generation."""
        m = archive.shape[0]
        if tuple(x.shape) != tuple(self.x.shape) or archive.shape[1] != self.d:
            raise BartmiError("state shapes do not match the sampler")
        if not 2 <= m <= self.z_cap:
            raise BartmiError("archive must hold 2..z_cap rows")
        self.x.copy_(x)
        self.z[:m].copy_(archive)
        self.counters.copy_(torch.tensor([generation, m], dtype=torch.int64))

    @property
    def generation(self) -> int:
        return int(self.counters[0])

    @property
    def archive_size(self) -> int:
        return int(self.counters[1])


class PerSampleForward:
    """The plain per-sample form of the forward model: one bm_forward_batch call per
    chain (B = 1), as BART runs one forward-model worker per chain, spread round-robin
    over ``workers`` streams with a workspace each. Same outputs as Forward(model, C,
    binned=True, chi2=True), written in place per sample."""

    def __init__(self, model, n_chains: int, workers: int = 1, device="cuda"):
        self.model, self.B, self.W = model, n_chains, workers
        self._structs = (BmModel * 1)(model.struct)
        self.n_nu, self.n_bins = model.n_nu, model.n_bins
        self.depth = torch.empty(n_chains * self.n_nu, dtype=torch.float64, device=device)
        self.binned = torch.empty(n_chains * self.n_bins, dtype=torch.float64, device=device)
        self.chi2 = torch.empty(n_chains, dtype=torch.float64, device=device)
        self.flags = torch.empty(n_chains, dtype=torch.int32, device=device)
        ws = int(lib().bm_workspace_size(self._structs, 1, None, 1))
        if ws == 0:
            raise BartmiError("bm_workspace_size rejected the model")
        self.ws_bytes = ws
        self.workspaces = [torch.zeros(ws, dtype=torch.uint8, device=device) for _ in range(workers)]
        self.streams = [torch.cuda.Stream() for _ in range(workers - 1)]

    def __call__(self, params: torch.Tensor, stream=None):
        if params.shape[0] != self.B or params.dtype != torch.float64 or not params.is_contiguous():
            raise BartmiError("params must be a contiguous float64 [B][P] device tensor")
        main = stream if stream is not None else torch.cuda.current_stream()
        streams = [main] + self.streams
        for s_ in self.streams:
            s_.wait_stream(main)
        P = params.shape[1]
        fn = lib().bm_forward_batch
        p0, d0, b0 = _ptr(params).value, _ptr(self.depth).value, _ptr(self.binned).value
        c0, f0 = _ptr(self.chi2).value, _ptr(self.flags).value
        wsp = [_ptr(w).value for w in self.workspaces]
        for c in range(self.B):
            w = c % self.W
            st = fn(self._structs, 1, None, C.c_void_p(p0 + 8 * P * c), P, 1, None,
                    C.c_void_p(d0 + 8 * self.n_nu * c),
                    C.c_void_p(b0 + 8 * self.n_bins * c) if self.n_bins else None,
                    C.c_void_p(c0 + 8 * c), C.c_void_p(f0 + 4 * c), C.c_void_p(wsp[w]),
                    C.c_size_t(self.ws_bytes), C.c_void_p(streams[w].cuda_stream))
            if st != 0:
                _check(st, "bm_forward_batch")
        for s_ in self.streams:
            main.wait_stream(s_)
        return self


class Retrieval:
    """A DE-MCz retrieval of one model's observation (model.data / model.err set).

    ``surrogate`` (optional) maps a [C][d] parameter tensor to a [C] surrogate chi^2 on
    the same stream; it enables two-stage delayed acceptance. ``per_sample_workers`` > 0
    selects the plain per-sample form (PerSampleForward) instead of one batched call per
    generation. ``p_snooker`` is the rate of snooker moves (DEMCzs; 0.1 as in ter Braak &
    Vrugt 2008). A parameter with lo = hi is held at that value (states and archive rows
    given to ``resume`` must hold it)."""

    def __init__(self, model, n_chains: int, lo, hi, seed: int, thin: int = 10,
                 hist_cap: int = 0, surrogate=None, eps_scale: float = 1e-6, z_cap=None,
                 per_sample_workers: int = 0, p_snooker: float = 0.1, gamma_scale: float = 1.0):
        self.model = model
        if per_sample_workers:
            if surrogate is not None:
                raise BartmiError("the per-sample form has no surrogate stage")
            self.fwd = PerSampleForward(model, n_chains, per_sample_workers)
        else:
            self.fwd = Forward(model, n_chains, binned=True, chi2=True)
        self.s = DEMCz(n_chains, lo, hi, seed, thin=thin, hist_cap=hist_cap, z_cap=z_cap,
                       eps_scale=eps_scale, surrogate=surrogate is not None, p_snooker=p_snooker,
                       gamma_scale=gamma_scale)
        self.surrogate = surrogate
        self.active = torch.ones(n_chains, dtype=torch.int32, device=self.s.x.device)

    def start(self, z_init: int | None = None):
        self.s.init(z_init)
        self._set_lp()

    def resume(self, x: torch.Tensor, archive: torch.Tensor):
        """Continue from given chain states and archive (e.g. after a burn-in)."""
        self.s.load_state(x, archive)
        self._set_lp()

    def reset_archive(self):
        """Replace the archive by the current chain states: drops the wide early states of
        a burn-in so that the difference vectors shrink to the current spread."""
        self.s.load_state(self.s.x.clone(), self.s.x.clone(), self.s.generation)
        self._set_lp()

    def _set_lp(self):
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

    def run_monitored(self, n_gen: int, burn: int = 0, n_saves: int = 10, chunk: int = 50,
                      checkpoint: str | None = None) -> dict:
        """Sec. 5's run cadence: the n_gen generations run in n_saves parts (whole graph
        replays of `chunk` generations); after each part the state can be saved
        (`checkpoint`, see save) and, once past the `burn` generations to discard, the
        Gelman-Rubin statistic of the kept samples is logged; at the end SPEIS and ESS of
        the kept samples. Needs a history buffer for every generation of the run."""
        from . import diagnostics as dg
        g0 = self.s.generation
        if self.s.history is None or self.s.history.shape[0] < g0 + n_gen:
            raise BartmiError("run_monitored needs a history of every generation")
        if n_gen % chunk or n_saves < 1:
            raise BartmiError("n_gen must be whole chunks")
        graph = self.capture(chunk)
        n_chunks = n_gen // chunk
        bounds = sorted({round(n_chunks * (i + 1) / n_saves) for i in range(n_saves)})
        log = []
        done = 0
        for b in bounds:
            for _ in range(b - done):
                graph.replay()
            done = b
            torch.cuda.synchronize()
            gen = self.s.generation
            if checkpoint:
                self.save(checkpoint)
            entry = {"generation": gen}
            if gen - g0 > burn + 1:
                kept = self.s.history[g0 + burn:gen].cpu().numpy()
                gr = dg.gelman_rubin(kept)
                entry.update(gr_max=float(np.max(gr)), gr=gr.tolist())
            log.append(entry)
        kept = self.s.history[g0 + burn:g0 + n_gen].cpu().numpy()
        sp = dg.speis_per_chain(kept)
        return {"log": log, "speis_max": float(sp.max()), "ess": float(kept.shape[0] * kept.shape[1] / sp.max()),
                "gelman_rubin": dg.gelman_rubin(kept).tolist()}

    def save(self, path: str):
        """Checkpoint of the sampler state (chains, archive, counters, log posteriors,
        acceptance counts, history) as a numpy archive of plain arrays."""
        s = self.s
        m = s.archive_size
        arrays = {"x": s.x, "z": s.z[:m], "counters": s.counters, "lp": s.lp, "n_accept": s.n_accept}
        if s.lp_surr is not None:
            arrays["lp_surr"] = s.lp_surr
        if s.history is not None:
            arrays["history"] = s.history[:min(s.generation, s.history.shape[0])]
        np.savez(path, **{k: v.cpu().numpy() for k, v in arrays.items()})

    def load(self, path: str):
        """Resume from a checkpoint written by save: the run continues with the same random
        stream (draws are addressed by generation), so it reproduces an uninterrupted run."""
        s = self.s
        with np.load(path, allow_pickle=False) as f:
            z = torch.as_tensor(f["z"], device=s.x.device)
            s.load_state(torch.as_tensor(f["x"], device=s.x.device), z, int(f["counters"][0]))
            s.lp.copy_(torch.as_tensor(f["lp"]))
            s.n_accept.copy_(torch.as_tensor(f["n_accept"]))
            if s.lp_surr is not None and "lp_surr" in f:
                s.lp_surr.copy_(torch.as_tensor(f["lp_surr"]))
            if s.history is not None and "history" in f:
                h = torch.as_tensor(f["history"])
                s.history[:h.shape[0]].copy_(h)

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


def fisher_covariance(model, theta, lo, hi, rel_step: float = 1e-4) -> np.ndarray:
    """Gaussian (Laplace) approximation of the posterior covariance at theta from the
    binned-spectrum Jacobian: (J^T diag(1/err^2) J + diag(12/width^2))^-1, J by central
    differences from one batched forward call of 2d + 1 spectra. The diagonal term is the
    variance of the uniform prior and keeps unconstrained directions at prior width."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    theta = np.asarray(theta, np.float64).ravel()
    d = theta.size
    width = hi - lo
    step = rel_step * width
    pts = np.repeat(theta[None], 2 * d + 1, axis=0)
    for j in range(d):
        pts[1 + 2 * j, j] += step[j]
        pts[2 + 2 * j, j] -= step[j]
    f = Forward(model, 2 * d + 1, binned=True)
    f(torch.as_tensor(pts, device=model.sigma.device))
    nb = model.n_bins
    y = f.binned.view(2 * d + 1, nb).cpu().numpy()
    if int((f.flags != 0).sum()):
        raise BartmiError("the forward model flagged a point of the Jacobian stencil")
    jac = np.stack([(y[1 + 2 * j] - y[2 + 2 * j]) / (2 * step[j]) for j in range(d)], axis=1)
    err = model.err.cpu().numpy()
    jw = jac / err[:, None]
    prec = jw.T @ jw + np.diag(12.0 / width ** 2)
    return np.linalg.inv(prec)


def gaussian_states(mean, cov, n: int, lo, hi, seed: int, inflate: float = 1.0) -> np.ndarray:
    """n draws from N(mean, inflate^2 cov), redrawn until inside the prior box."""
    g = np.random.default_rng(seed)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    chol = np.linalg.cholesky(cov) * inflate
    out = np.empty((0, lo.size))
    while out.shape[0] < n:
        x = np.asarray(mean, np.float64)[None] + g.normal(size=(2 * n, lo.size)) @ chol.T
        x = x[np.all((x >= lo) & (x <= hi), axis=1)]
        out = np.vstack([out, x])
    return out[:n]
