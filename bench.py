"""Benchmark of the transmission forward model and the retrieval built on it, one MI355X.

Headline (``forward``): the full single forward model, one spectrum per call, back to
back on one stream. 4 absorbers with opacity tables on 20 temperatures (300-3000 K) x
100 log-spaced layers (1e-8--100 bar) x 30000 wavenumbers (0.5 cm^-1 from 1000 cm^-1) in
float32, built by the library's line-by-line opacity build (1e5-1e6 synthetic lines per
absorber), a 20 x 30000 H2-H2 CIA table, the five-parameter T(p) profile. A step is one
bm_forward_batch call with B = 1: atmosphere, extinction, chord optical depth, transit
depth (a1-a5), 30-point channels and chi^2 against a synthetic observation (a6); every
step uses a different prior draw. ``roofline`` is for the fused kernel, timed per launch
with HIP events on its stream (bm_timing_start/stop).

Further sections, each reported in its own object of the same JSON line:
  batched   256 DE-MCz chains per generation in one graph-captured launch sequence, and a
            mixed batch of three instances (60/100/150 layers, 8000/30000/50000
            wavenumbers) fused in one launch; launch configurations autotuned.
  mcmc      the learned surrogate (MLP 10 -> 4 x 512 -> 1000, BF16) trained on forward-model
            spectra, as stage 1 of delayed acceptance in 256-chain DE-MCz, against the
            plain per-sample forward model: effective samples/s and posterior agreement.
  opacity   the line-by-line opacity-table build, 1e7 lines onto 1e5 wavenumbers x 20 T x
            100 p (opt-in: --sections ...,opacity).
Inputs are resident in HBM before any timed region. One JSON line goes to stdout;
progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

T_START = time.time()

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0   # dense matrix cores


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ----------------------------------------------------------------------------- inputs
def device_lines(lines):
    """The line list's arrays as device tensors (resident in HBM before a timed build)."""
    import torch
    import workloads as wl
    return wl.LineList(*(torch.as_tensor(np.ascontiguousarray(getattr(lines, f)), device="cuda")
                         for f in ("nu0", "s296", "gamma296", "elow", "mass_amu")))


def build_tables(setup, how: str, seed: int):
    import torch
    import workloads as wl
    import paper_2104_12522_amd as bm
    S, L, N = setup.n_species, setup.p_bar.size, setup.nu.size
    if how == "random":
        sig = wl.random_opacity_table(S, setup.temps, L, setup.nu, seed=seed, dtype=np.float32)
        return torch.as_tensor(sig, device="cuda")
    out = torch.empty(S, len(setup.temps), L, N, dtype=torch.float32, device="cuda")
    for i, n_lines in enumerate(setup.lines_per_species):
        lines = wl.line_list(n_lines, seed=seed + i, mass_amu=float(setup.mass_amu[i]))
        t0 = time.time()
        bm.opacity_table_build(lines, setup.temps, setup.p_bar, float(setup.nu[0]),
                               float(setup.nu[1] - setup.nu[0]), N, out=out[i])
        torch.cuda.synchronize()
        log(f"opacity table {setup.name} species {i}: {n_lines} lines in {time.time() - t0:.2f} s")
    return out


def make_model(setup, sigma, seed: int, truth=None):
    """Model of one setup with a synthetic observation: the forward model at `truth` (a
    prior draw when None) binned to 30-point channels plus 60 ppm Gaussian noise."""
    import torch
    import workloads as wl
    import paper_2104_12522_amd as bm
    cia = torch.as_tensor(wl.cia_table(setup.cia_temps, setup.nu), device="cuda")
    nb = setup.nu.size // setup.bin_width
    model = bm.Model(sigma, setup.temps, setup.p_bar, setup.mass_amu, setup.tp_mode,
                     setup.planet, cia=cia, cia_temps=setup.cia_temps,
                     bin_width=setup.bin_width, data=np.zeros(nb), err=np.full(nb, 60e-6))
    prior = wl.line2013_prior(setup.n_species)
    if truth is None:
        truth = prior.draw(1, seed=seed + 2)[0]
    # two copies of the truth: no section tunes a two-spectrum call, so the observation
    # takes the default launch configuration whichever sections ran before (the pipelined
    # configuration that a tuned one-spectrum call may use sums the chord depths in another
    # order, which moves the observation in its last bits and with it every chain)
    f = bm.Forward(model, 2, binned=True)
    f(torch.as_tensor(np.repeat(np.asarray(truth, np.float64)[None], 2, axis=0), device="cuda"))
    noise = wl.rng(seed + 3).normal(0.0, 60e-6, nb)
    model.set_observation(f.binned_spectrum(0).cpu().numpy() + noise, np.full(nb, 60e-6))
    return model, cia


def spectrum_bytes(S, L, N, NTC, nb):
    """Algorithmic HBM bytes of one spectrum: the two bracketing temperature rows of every
    species table on every layer (float32), the CIA table once (double), the spectrum and
    the channel means out (double)."""
    return 4 * (2 * S * L * N) + 8 * NTC * N + 8 * N + 8 * nb


def spectrum_flops(S, L, N):
    """Algorithmic FP32 operations of one spectrum: the temperature interpolation and
    density weighting (4 per species, layer and wavenumber), the chord optical depths
    (2 per nonzero chord weight), 1 - exp(-tau) and the impact-parameter sum (~4 per
    chord and wavenumber)."""
    return N * (4 * S * L + L * (L + 1) + 4 * L)


def traffic_from_profile(workload: str, config: int):
    """HBM bytes per launch of the fused kernel (counter runs summarised in
    profiles/forward_traffic.json) for a workload and launch configuration, or None when
    the kernel source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "forward_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, rec["kernel_source"]), "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    if rec.get("kernel_sha256") != digest:
        return None
    entry = rec["workloads"].get(workload, {}).get("configs", {}).get(str(config))
    return None if entry is None else entry["hbm_bytes_per_launch"]


# ----------------------------------------------------------------------------- sections
def section_forward(args, setup, model, prior):
    """Headline: one spectrum per call on one stream."""
    import torch
    import paper_2104_12522_amd as bm
    S, L, N = setup.n_species, setup.p_bar.size, setup.nu.size
    NTC, nb = len(setup.cia_temps), N // setup.bin_width
    n_draw = args.warmup + args.steps
    params = torch.as_tensor(prior.draw(n_draw, seed=args.seed + 1), device="cuda").contiguous()
    rows = [params[i:i + 1] for i in range(n_draw)]
    f = bm.Forward(model, 1, binned=True, chi2=True)
    tuned, times = f.tune(rows[0], reps=50)
    cfg_names = bm.forward_configs()
    log(f"forward: autotuned one-spectrum call -> config {tuned} ({cfg_names[tuned]}); us per call "
        f"{[round(t * 1e3, 1) for t in times]}")
    # The tuner repeats one parameter set, so every repetition reads the same table rows;
    # the timed loop draws new parameters for each call, which read rows that the 256 MB
    # Infinity Cache holds only in part (the tables are 960 MB). Its two best candidates
    # are timed again that way (300 calls each, two interleaved rounds) and the faster kept.
    cands = [c for _, c in sorted((t, c) for c, t in enumerate(times) if t > 0)[:2]]
    steady = {c: 0.0 for c in cands}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        for c in cands:
            f.set_config(c)
            f(rows[0])
            e0.record()
            for i in range(300):
                f(rows[i % n_draw])
            e1.record()
            torch.cuda.synchronize()
            steady[c] += e0.elapsed_time(e1) / 600
    chosen = min(steady, key=steady.get)
    f.set_config(chosen)
    log(f"forward: varied-parameter check of configs {cands}: us per call "
        f"{[round(steady[c] * 1e3, 2) for c in cands]} -> config {chosen} ({cfg_names[chosen]})")
    for i in range(args.warmup):
        f(rows[i])
    torch.cuda.synchronize()
    log(f"forward: warmup {args.warmup} done, timing {args.steps} one-spectrum calls")
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    t0 = time.perf_counter()
    for i in range(args.steps):
        f(rows[args.warmup + i])
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end) / args.steps
    # the fused kernel alone: the same calls again, each kernel launch between two events,
    # after a run-in of untimed calls that keeps the GPU busy while the host sets up the
    # events (so that a short pass is not timed from an idle GPU)
    for i in range(max(args.warmup, 100)):
        f(rows[i % n_draw])
    with bm.KernelTiming(args.steps) as kt:
        for i in range(args.steps):
            f(rows[args.warmup + i])
        torch.cuda.synchronize()
    log(f"forward: {ms * 1e3:.2f} us per spectrum (events), {wall / args.steps * 1e6:.2f} us (host "
        f"clock); fused kernel {kt.mean_ms * 1e3:.2f} us over {kt.launches} launches")
    bytes_spec = spectrum_bytes(S, L, N, NTC, nb)
    achieved = bytes_spec / (kt.mean_ms * 1e-3) / 1e9
    traffic = traffic_from_profile("config2_b1", chosen)
    out = {
        "ms_per_step": ms,
        "value": 1000.0 / ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_forward (fused extinction, chord optical depth, depth, channels)",
                     "bytes_per_launch": bytes_spec, "kernel_us": kt.mean_ms * 1e3,
                     "launches_timed": kt.launches,
                     "call_us": ms * 1e3,
                     "call_frac": bytes_spec / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "last_flags": int(f.flags[0]),
        "autotune": {"chosen": chosen, "tuner_choice": tuned, "configs": cfg_names, "ms_per_call": times,
                     "varied_check_ms_per_call": {str(c): steady[c] for c in cands}},
    }
    if args.workers > 1:
        out["multi_worker"] = multi_worker(args, model, rows)
    return out


def section_fp64(args):
    """The FP64 single-spectrum workload: one absorber with 1e4 lines, its table built by
    the library in double (10 T x 50 p x 1000 nu at 4 cm^-1), an isothermal 1200 K
    atmosphere with x = 1e-4; one spectrum per call, back to back on one stream. Latency
    per spectrum from HIP events, and the fused kernel's own time."""
    import torch
    import workloads as wl
    import paper_2104_12522_amd as bm
    s = wl.config1()
    lines = device_lines(wl.line_list(s.lines_per_species[0], seed=wl.SEED_BASE + 1,
                                      mass_amu=float(s.mass_amu[0])))
    dnu = float(s.nu[1] - s.nu[0])
    table = bm.opacity_table_build(lines, s.temps, s.p_bar, float(s.nu[0]), dnu, s.nu.size,
                                   dtype=torch.float64)
    model = bm.Model(table.reshape(1, *table.shape).contiguous(), s.temps, s.p_bar, s.mass_amu,
                     s.tp_mode, s.planet)
    n = args.warmup + args.steps
    draws = np.array([wl.config1_params()] * n)        # isothermal 1200 K, x = 1e-4
    params = torch.as_tensor(draws, device="cuda").contiguous()
    rows = [params[i:i + 1] for i in range(n)]
    f = bm.Forward(model, 1)
    for i in range(args.warmup):
        f(rows[i])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(args.steps):
        f(rows[args.warmup + i])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    with bm.KernelTiming(args.steps) as kt:
        for i in range(args.steps):
            f(rows[args.warmup + i])
        torch.cuda.synchronize()
    # algorithmic bytes: two temperature rows per layer (double), the spectrum out
    nbytes = 8 * (2 * s.p_bar.size * s.nu.size) + 8 * s.nu.size
    log(f"fp64 single spectrum: {ms * 1e3:.2f} us per call, fused kernel {kt.mean_ms * 1e3:.2f} us")
    return {"workload": "FP64, 1 absorber (1e4 lines, library-built double table), 10 T x 50 layers "
                        "x 1000 nu, isothermal, 1 spectrum per call on one stream",
            "us_per_spectrum": ms * 1e3, "spectra_per_s": 1000.0 / ms, "kernel_us": kt.mean_ms * 1e3,
            "bytes_per_launch": nbytes, "kernel_gbs": nbytes / (kt.mean_ms * 1e-3) / 1e9,
            "steps": args.steps}


def multi_worker(args, model, rows):
    """BART's layout: one forward-model worker per chain, here W concurrent streams each
    issuing one-spectrum calls (step i on worker i mod W)."""
    import torch
    import paper_2104_12522_amd as bm
    W = args.workers
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(W - 1)]
    fwds = [bm.Forward(model, 1, binned=True, chi2=True) for _ in range(W)]
    for i in range(args.warmup):
        fwds[i % W](rows[i], stream=streams[i % W])
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    main = streams[0]
    start.record(main)
    for s_ in streams[1:]:
        s_.wait_event(start)
    for i in range(args.steps):
        fwds[i % W](rows[args.warmup + i], stream=streams[i % W])
    for s_ in streams[1:]:
        ev = torch.cuda.Event()
        ev.record(s_)
        main.wait_event(ev)
    end.record(main)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / args.steps
    log(f"forward, {W} workers: {ms * 1e3:.2f} us per spectrum")
    return {"workers": W, "value": 1000.0 / ms, "ms_per_step": ms}


def graph_time(fn, n_inner: int, n_replay: int):
    """Capture fn() n_inner times in a HIP graph on a side stream, replay it n_replay
    times; returns ms per fn() from events around the replays."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            for _ in range(n_inner):
                fn()
    torch.cuda.current_stream().wait_stream(side)
    g.replay()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(n_replay):
        g.replay()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / (n_inner * n_replay)


def section_batched(args, setup, model, prior):
    """256 chains per DE-MCz generation, graph-captured; mixed-instance batch."""
    import torch
    import workloads as wl
    import paper_2104_12522_amd as bm
    from paper_2104_12522_amd.mcmc import Retrieval
    S, L, N = setup.n_species, setup.p_bar.size, setup.nu.size
    NTC, nb = len(setup.cia_temps), N // setup.bin_width
    C = args.chains
    cfg_names = bm.forward_configs()
    r = Retrieval(model, C, prior.lo, prior.hi, seed=args.seed + 20, thin=10,
                  z_cap=10 * prior.lo.size + C * (args.batched_gens // 10 + 20))
    r.start()
    chosen, times = r.fwd.tune(r.s.x.contiguous(), reps=3)
    log(f"batched: autotuned {C}-chain forward -> config {chosen} ({cfg_names[chosen]}); "
        f"ms per call {[round(t, 3) for t in times]}")
    r.start()
    # forward only: one B = C call per graph node, replayed
    x = r.s.x.contiguous()
    ms_fwd = graph_time(lambda: r.fwd(x), 10, max(1, args.batched_gens // 10))
    with bm.KernelTiming(20) as kt:
        for _ in range(20):
            r.fwd(x)
        torch.cuda.synchronize()
    bytes_gen = C * spectrum_bytes(S, L, N, NTC, nb)
    flops_gen = C * spectrum_flops(S, L, N)
    # whole generations (propose, forward, accept) captured in one graph
    r.start()
    ms_gen = graph_time(r.generation, 10, max(1, args.batched_gens // 10))
    log(f"batched: {ms_fwd:.3f} ms per {C}-spectrum forward call, {ms_gen:.3f} ms per generation, "
        f"fused kernel {kt.mean_ms:.3f} ms")
    out = {
        "chains": C,
        "autotune": {"chosen": chosen, "configs": cfg_names, "ms_per_call": times},
        "forward_ms_per_call": ms_fwd,
        "spectra_per_s": C / (ms_fwd * 1e-3),
        "generation_ms": ms_gen,
        "generation_spectra_per_s": C / (ms_gen * 1e-3),
        "kernel_ms": kt.mean_ms,
        "hbm_equiv": {"achieved": bytes_gen / (kt.mean_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "note": "algorithmic bytes as if every spectrum streamed "
                                              "its table rows from HBM; chains of a tile share "
                                              "rows through L2"},
        "fp32": {"achieved": flops_gen / (kt.mean_ms * 1e-3) / 1e12, "peak": FP32_PEAK_TFLOPS,
                 "unit": "TFLOP/s"},
        "traffic": traffic_from_profile("config2_b256", chosen),
    }
    if args.mixed:
        out["mixed"] = section_mixed(args, prior)
    return out


def section_mixed(args, prior):
    import torch
    import workloads as wl
    import paper_2104_12522_amd as bm
    setups = wl.config3_mixed()
    models = []
    for k, s in enumerate(setups):
        sig = build_tables(s, args.table, args.seed + 100 * (k + 1))
        m, _ = make_model(s, sig, args.seed + 100 * (k + 1))
        models.append(m)
    C = args.chains
    inst = [min(k * len(setups) // C, len(setups) - 1) for k in range(C)]   # contiguous thirds
    params = torch.as_tensor(prior.draw(C, seed=args.seed + 30), device="cuda").contiguous()
    f = bm.Forward(models, C, instance=inst, binned=True, chi2=True)
    chosen, times = f.tune(params, reps=3)
    ms = graph_time(lambda: f(params), 5, 10)
    with bm.KernelTiming(10) as kt:
        for _ in range(10):
            f(params)
        torch.cuda.synchronize()
    bytes_call = sum(spectrum_bytes(s.n_species, s.p_bar.size, s.nu.size, len(s.cia_temps),
                                    s.nu.size // s.bin_width) for s in (setups[i] for i in inst))
    log(f"mixed batch: {ms:.3f} ms per call of {C} spectra over {len(setups)} instances "
        f"(config {chosen}); fused kernel {kt.mean_ms:.3f} ms")
    return {"instances": [{"n_layers": int(s.p_bar.size), "n_nu": int(s.nu.size),
                           "dnu": float(s.nu[1] - s.nu[0]), "samples": int(inst.count(k))}
                          for k, s in enumerate(setups)],
            "launches_per_call": 1, "ms_per_call": ms, "spectra_per_s": C / (ms * 1e-3),
            "kernel_ms": kt.mean_ms,
            "hbm_equiv_gbs": bytes_call / (kt.mean_ms * 1e-3) / 1e9,
            "autotune": {"chosen": chosen, "ms_per_call": times}}


def section_mcmc(args, setup, prior):
    """Learned surrogate + delayed acceptance against the plain per-sample forward model."""
    import torch
    import paper_2104_12522_amd as bm
    from paper_2104_12522_amd import diagnostics as dg
    from paper_2104_12522_amd.mcmc import (Retrieval, fisher_covariance, gaussian_states)
    from paper_2104_12522_amd.surrogate import (MLP, Surrogate, Trainer, standardisation,
                                                training_set)
    sigma = args._sigma
    truth = np.array([-1.5, -0.6, 0.2, 0.3, 0.9, -3.5, -4.0, -5.0, -6.0, 1.15])
    model, _ = make_model(setup, sigma, args.seed + 50, truth=truth)
    C, G, BURN = args.chains, args.mcmc_gens, args.mcmc_burn
    nb = model.n_bins
    d = prior.lo.size
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")  # noqa: E731
    lo_p, hi_p = dev(prior.lo), dev(prior.hi)

    def run_graph(r, n_gen, chunk=50):
        g_ = r.capture(chunk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n_gen // chunk):
            g_.replay()
            if i % 40 == 39:
                torch.cuda.synchronize()
                log(f"mcmc: {(i + 1) * chunk} / {n_gen} generations")
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def train(net, lo, hi, X, Y, mean, scale, epochs, lr0, seed):
        tr = Trainer(net, lo, hi, X, Y, mean, scale, batch=512, seed=seed)
        for e in range(epochs):
            tr.epoch(1e-6 + 0.5 * (lr0 - 1e-6) * (1 + math.cos(math.pi * e / epochs)))

    def spectra(xs):
        n = xs.shape[0]
        Y = torch.empty(n, nb, dtype=torch.float64, device="cuda")
        fw = None
        for s0 in range(0, n, 4096):
            m = min(4096, n - s0)
            if fw is None or fw.B != m:
                fw = bm.Forward(model, m, binned=True)
            fw(xs[s0:s0 + m].contiguous())
            Y[s0:s0 + m] = fw.binned.view(m, nb)
        return Y

    def rms_ppm(sur, xs, ys):
        pred = sur.mean + sur.scale * sur.predict(xs).double()
        return float(torch.sqrt(((pred - ys) ** 2).mean())) * 1e6

    # 1. surrogate on prior draws (2e5 spectra from the forward model)
    t0 = time.perf_counter()
    X, Y = training_set(model, prior, args.train_spectra + 5000, seed=args.seed + 60)
    Xte, Yte = X[-5000:].contiguous(), Y[-5000:].contiguous()
    X, Y = X[:-5000].contiguous(), Y[:-5000].contiguous()
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    mean, scale = standardisation(Y)
    dims = [d, 512, 512, 512, 512, nb]
    net = MLP(dims, max_batch=5000, seed=1)
    t0 = time.perf_counter()
    train(net, lo_p, hi_p, X, Y, mean, scale, args.epochs, 1e-3, 2)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    sur_p = Surrogate(net, lo_p, hi_p, mean, scale, model.data, model.err, n_chains=5000)
    rms_prior = rms_ppm(sur_p, Xte, Yte)
    log(f"mcmc: prior surrogate: {X.shape[0]} spectra in {t_data:.1f} s, {args.epochs} epochs in "
        f"{t_train:.1f} s ({net.step} Adam steps), held-out rms {rms_prior:.2f} ppm")
    del X, Y

    # launch configuration of the C-chain forward call, tuned once for every run below
    tune_fwd = bm.Forward(model, C, binned=True, chi2=True)
    chosen, _ = tune_fwd.tune(dev(prior.draw(C, seed=args.seed + 66)), reps=8)
    log(f"mcmc: {C}-chain forward call tuned -> config {chosen}")
    del tune_fwd

    # 2. burn-in with the exact sampler from the Laplace approximation at the truth
    cov = fisher_covariance(model, truth, prior.lo, prior.hi)
    x_init = dev(gaussian_states(truth, cov, C, prior.lo, prior.hi, seed=args.seed + 61))
    z_init = dev(gaussian_states(truth, cov, 10 * C, prior.lo, prior.hi, seed=args.seed + 62))
    rb = Retrieval(model, C, prior.lo, prior.hi, seed=args.seed + 63, thin=10, hist_cap=BURN,
                   z_cap=10 * C + C * (BURN // 10 + 2))
    rb.resume(x_init, z_init)
    t_burn = run_graph(rb, BURN)
    hb = rb.s.history[BURN // 2:BURN].cpu().numpy().reshape(-1, d)
    mu_b, cov_b = hb.mean(0), np.cov(hb.T)
    sd_b = np.sqrt(np.diag(cov_b))
    x0 = rb.s.x.clone()
    m = rb.s.archive_size
    z0 = rb.s.z[max(0, m - 10 * C):m].clone()
    log(f"mcmc: burn-in {BURN} generations in {t_burn:.1f} s")
    post_np = hb[np.random.default_rng(args.seed + 64).choice(hb.shape[0], 2048, replace=False)]
    post_x = dev(post_np)
    post_y = spectra(post_x)
    rms_prior_post = rms_ppm(sur_p, post_x, post_y)

    # 3. local surrogate: inputs on a +-5 sd box around the burn-in states, outputs
    #    standardised on spectra drawn around them (BF16 inputs resolve ~1/256 of the box)
    t0 = time.perf_counter()
    lo_l = np.maximum(mu_b - args.surrogate_box * sd_b, prior.lo)
    hi_l = np.minimum(mu_b + args.surrogate_box * sd_b, prior.hi)
    Xl = dev(gaussian_states(mu_b, cov_b, args.local_spectra, lo_l, hi_l, seed=args.seed + 65,
                             inflate=2.0))
    Yl = spectra(Xl)
    mean_l, scale_l = standardisation(Yl)
    net_l = MLP(dims, max_batch=5000, seed=3)
    train(net_l, dev(lo_l), dev(hi_l), Xl, Yl, mean_l, scale_l, args.epochs, 1e-3, 4)
    torch.cuda.synchronize()
    t_local = time.perf_counter() - t0
    sur = Surrogate(net_l, dev(lo_l), dev(hi_l), mean_l, scale_l, model.data, model.err,
                    n_chains=5000)
    rms_local = rms_ppm(sur, post_x, post_y)
    fw = bm.Forward(model, C, binned=True, chi2=True)
    fw(post_x[:C].contiguous())
    dchi2 = (sur(post_x[:C].contiguous()) - fw.chi2).cpu().numpy()
    log(f"mcmc: local surrogate in {t_local:.1f} s; rms near the posterior: prior-trained "
        f"{rms_prior_post:.2f} ppm, local {rms_local:.2f} ppm")
    del Xl, Yl

    # the surrogate's matrix-core work: one C-chain inference (input scaling, five BF16
    # products with fused epilogues, chi^2) timed with events; training steps from the
    # prior surrogate's training wall time
    xs = post_x[:C].contiguous()
    sur(xs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(200):
        sur(xs)
    e1.record()
    torch.cuda.synchronize()
    us_inf = e0.elapsed_time(e1) / 200 * 1e3
    macs = sum(dims[i] * dims[i + 1] for i in range(len(dims) - 1))
    fl_inf = 2.0 * C * macs
    # a training step: forward (2 B macs), weight gradients (2 B macs) and input gradients
    # of every layer but the first (2 B macs each)
    fl_step = 2.0 * 512 * (3 * macs - dims[0] * dims[1])
    mfma = {"inference_us_per_call": us_inf, "inference_gflop": fl_inf / 1e9,
            "inference_tflops": fl_inf / (us_inf * 1e-6) / 1e12,
            "train_step_us": t_train / max(net.step, 1) * 1e6, "train_step_gflop": fl_step / 1e9,
            "train_tflops": fl_step * net.step / t_train / 1e12, "peak_tflops": BF16_PEAK_TFLOPS}
    mfma["inference_frac"] = mfma["inference_tflops"] / BF16_PEAK_TFLOPS
    mfma["train_frac"] = mfma["train_tflops"] / BF16_PEAK_TFLOPS
    log(f"mcmc: surrogate inference {us_inf:.1f} us per {C}-chain call ({mfma['inference_tflops']:.1f} "
        f"TFLOP/s), training {mfma['train_tflops']:.1f} TFLOP/s (BF16 peak {BF16_PEAK_TFLOPS:.0f})")

    # 3b. longer burn-in with delayed acceptance (exact, and cheap), then the local
    #     surrogate is refit to the wider set of states
    if args.da_burn > 0:
        rd = Retrieval(model, C, prior.lo, prior.hi, seed=args.seed + 67, thin=10, hist_cap=args.da_burn,
                       surrogate=sur, z_cap=z0.shape[0] + C * (args.da_burn // 10 + 2))
        rd.resume(x0, z0)
        t_db = run_graph(rd, args.da_burn)
        hb = rd.s.history[args.da_burn // 2:args.da_burn].cpu().numpy().reshape(-1, d)
        mu_b, cov_b = hb.mean(0), np.cov(hb.T)
        sd_b = np.sqrt(np.diag(cov_b))
        x0 = rd.s.x.clone()
        m = rd.s.archive_size
        z0 = rd.s.z[max(0, m - 10 * C):m].clone()
        t0 = time.perf_counter()
        lo_l = np.maximum(mu_b - args.surrogate_box * sd_b, prior.lo)
        hi_l = np.minimum(mu_b + args.surrogate_box * sd_b, prior.hi)
        Xl = dev(gaussian_states(mu_b, cov_b, args.local_spectra, lo_l, hi_l, seed=args.seed + 68,
                                 inflate=2.0))
        Yl = spectra(Xl)
        mean_l, scale_l = standardisation(Yl)
        net_l = MLP(dims, max_batch=5000, seed=7)
        train(net_l, dev(lo_l), dev(hi_l), Xl, Yl, mean_l, scale_l, args.epochs, 1e-3, 8)
        torch.cuda.synchronize()
        t_local += time.perf_counter() - t0
        sur = Surrogate(net_l, dev(lo_l), dev(hi_l), mean_l, scale_l, model.data, model.err,
                        n_chains=5000)
        post_np = hb[np.random.default_rng(args.seed + 69).choice(hb.shape[0], 2048, replace=False)]
        post_x = dev(post_np)
        post_y = spectra(post_x)
        rms_local = rms_ppm(sur, post_x, post_y)
        fw(post_x[:C].contiguous())
        dchi2 = (sur(post_x[:C].contiguous()) - fw.chi2).cpu().numpy()
        log(f"mcmc: delayed-acceptance burn-in {args.da_burn} generations in {t_db:.1f} s; local "
            f"surrogate refit, rms {rms_local:.2f} ppm")
        del Xl, Yl

    # 4. production runs from the burned-in state, each on its own random stream: two plain
    #    batched runs (the second is the plain sampler's own run-to-run yardstick) and a
    #    longer delayed-acceptance run
    G_da = args.da_gens
    # the two plain runs are shortened (to whole thousands of generations) when the rates
    # measured in burn-in say that the whole run would not fit its time budget
    s_gen = t_burn / BURN
    s_gen_da = t_db / args.da_burn if args.da_burn > 0 else 0.3e-3
    G_f = args.fixed_tp_gens
    # what the sections after the plain runs take: the delayed-acceptance run, the T(p)-fixed
    # runs (two plain runs and a burn-in at the plain rate; two delayed-acceptance runs of
    # 5 G_f generations that cost about 0.31 and 0.13 of a plain generation there, where a
    # fifth and a thirteenth of the proposals pass the surrogate), the opacity section, with
    # a 20 % margin
    reserve = (20.0 + 1.2 * G_da * s_gen_da + (30.0 if "opacity" in args._sections else 0.0)
               + (1.2 * ((2 * G_f + args.fixed_tp_burn) + 5 * G_f * (0.31 + 0.13)) * s_gen + 15.0
                  if G_f > 0 else 0.0))
    left = args.time_budget - (time.time() - args._t0) - reserve
    G_asked = G
    if 2 * G * s_gen > left:
        G = max(5000, int(left / (2 * s_gen)) // 1000 * 1000)
        log(f"mcmc: plain runs shortened to {G} generations ({left:.0f} s of the time budget left)")
    def production(surrogate=None, per_sample=0, n_gen=G, stream=70):
        r = Retrieval(model, C, prior.lo, prior.hi, seed=args.seed + stream, thin=10, hist_cap=n_gen,
                      surrogate=surrogate, per_sample_workers=per_sample,
                      z_cap=z0.shape[0] + C * (n_gen // 10 + 1))
        r.resume(x0, z0)
        torch.cuda.synchronize()
        if per_sample:
            t0_ = time.perf_counter()
            r.run(n_gen)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0_
        else:
            wall = run_graph(r, n_gen)
        h = r.s.history[:n_gen]
        acc = r.s.n_accept.sum(0).cpu().numpy() / (C * n_gen)
        return r, h, wall, acc

    def stats(h, wall, acc, n_gen, **extra):
        hn = h.cpu().numpy()
        sp = dg.speis_per_chain(hn)
        ess = hn.shape[0] * hn.shape[1] / sp.max()
        # the multi-chain integrated time, on every 10th state of long runs (scaled back)
        th = 10 if n_gen > 40000 else 1
        tau = dg.integrated_time_multichain(hn[::th]) * th
        ess_mc = hn.shape[0] * hn.shape[1] / tau
        mu, sd = dg.marginal_summary(hn)
        out = {"generations": n_gen, "wall_s": wall, "ms_per_generation": wall / n_gen * 1e3,
               "acceptance": float(acc[1]), "speis_max": float(sp.max()),
               "speis_median": float(np.median(sp)), "ess": float(ess),
               "ess_per_s": float(ess / wall),
               "integrated_time_multichain": tau.tolist(),
               "ess_multichain_min": float(ess_mc.min()),
               "ess_multichain_per_s": float(ess_mc.min() / wall),
               "gelman_rubin_max": float(dg.gelman_rubin(hn).max())}
        out.update(extra)
        return out, mu, sd, tau

    log(f"mcmc: plain batched production, {G} generations")
    _, h_b, w_b, acc_b = production(stream=70)
    plain_b, mu_b2, sd_b2, tau_b = stats(h_b, w_b, acc_b, G)
    log(f"mcmc: plain batched replicate (another random stream), {G} generations")
    _, h_q, w_q, acc_q = production(stream=72)
    plain_q, mu_q, sd_q, tau_q = stats(h_q, w_q, acc_q, G)
    del h_q
    log(f"mcmc: delayed-acceptance production, {G_da} generations")
    _, h_d, w_d, acc_d = production(surrogate=sur, n_gen=G_da, stream=71)
    da, mu_d, sd_d, tau_d = stats(h_d, w_d, acc_d, G_da, stage1_pass_rate=float(acc_d[0]))
    # the same run over its first G generations: equal length and start as the plain runs
    mu_d_g = h_d[:G].reshape(-1, d).mean(0).cpu().numpy()
    del h_d
    mu_start = x0.mean(0).cpu().numpy()
    log(f"mcmc: plain per-sample, {args.per_sample_gens} generations timed")
    _, h_p, w_p, _ = production(per_sample=1, n_gen=args.per_sample_gens)
    identical = bool(torch.equal(h_p, h_b[:args.per_sample_gens]))
    del h_b
    ms_ps = w_p / args.per_sample_gens * 1e3
    # the per-sample form computes the same chains (checked above on the timed slice), so
    # its effective samples over G generations are the batched plain run's
    ps_wall = ms_ps * 1e-3 * G
    plain_ps = {"ms_per_generation": ms_ps, "timed_generations": args.per_sample_gens,
                "chains_identical_to_batched": identical, "ess": plain_b["ess"],
                "ess_per_s": plain_b["ess"] / ps_wall,
                "ess_multichain_min": plain_b["ess_multichain_min"],
                "ess_multichain_per_s": plain_b["ess_multichain_min"] / ps_wall}
    # posterior agreement: marginal means in units of the posterior sd (pooled plain runs),
    # with the Monte Carlo standard error of each run's mean from its integrated time
    sd_ref = 0.5 * (sd_b2 + sd_q)
    mu_plain = 0.5 * (mu_b2 + mu_q)
    se = lambda tau, n: sd_ref * np.sqrt(tau / (n * C))  # noqa: E731
    se_plain = 0.5 * np.sqrt(se(tau_b, G) ** 2 + se(tau_q, G) ** 2)
    diff = (mu_d - mu_plain) / sd_ref
    diff_se = np.sqrt(se_plain ** 2 + se(tau_d, G_da) ** 2) / sd_ref
    diff_pp = (mu_q - mu_b2) / sd_ref
    diff_eq = (mu_d_g - mu_plain) / sd_ref
    diff_pp_se = np.sqrt(se(tau_b, G) ** 2 + se(tau_q, G) ** 2) / sd_ref
    ratio = da["ess_per_s"] / plain_ps["ess_per_s"]
    ratio_mc = da["ess_multichain_per_s"] / plain_ps["ess_multichain_per_s"]
    # end to end: surrogate data and training charged to the delayed-acceptance run
    e2e = (da["ess_multichain_min"] / (w_d + t_local)) / plain_ps["ess_multichain_per_s"]
    fixed_tp = (section_fixed_tp(args, model, prior, truth, cov, C, run_graph, stats, ms_ps, spectra,
                                 train, dims) if G_f > 0 else None)
    log(f"mcmc: ESS/s per-sample {plain_ps['ess_per_s']:.2f}, batched {plain_b['ess_per_s']:.2f}, "
        f"delayed acceptance {da['ess_per_s']:.2f} -> {ratio:.1f}x (multi-chain ESS: {ratio_mc:.1f}x); "
        f"max |mean diff| delayed acceptance vs plain {np.abs(diff).max():.3f} sd "
        f"(first {G} generations {np.abs(diff_eq).max():.3f} sd; plain vs plain {np.abs(diff_pp).max():.3f} sd)")
    return {
        "chains": C, "burn_in": BURN, "da_burn_in": args.da_burn, "truth": truth.tolist(),
        "plain_generations_asked": G_asked, "time_budget_s": args.time_budget,
        "prior": {"lo": prior.lo.tolist(), "hi": prior.hi.tolist()},
        "surrogate": {"dims": dims, "dtype": "bf16 weights/activations, fp32 accumulate",
                      "train_spectra": args.train_spectra, "epochs": args.epochs,
                      "data_s": t_data, "train_s": t_train, "adam_steps": net.step,
                      "rms_ppm_prior_heldout": rms_prior, "matrix_cores": mfma,
                      "rms_ppm_near_posterior": rms_prior_post,
                      "local": {"train_spectra": args.local_spectra, "s": t_local,
                                "rms_ppm_near_posterior": rms_local,
                                "chi2_error_mean": float(dchi2.mean()),
                                "chi2_error_sd": float(dchi2.std())}},
        "plain_per_sample": plain_ps,
        "plain_batched": plain_b,
        "plain_batched_replicate": plain_q,
        "delayed_acceptance": da,
        "ess_per_s_ratio_vs_per_sample": ratio,
        "ess_multichain_per_s_ratio_vs_per_sample": ratio_mc,
        "ess_per_s_ratio_vs_batched": da["ess_per_s"] / plain_b["ess_per_s"],
        "ess_multichain_per_s_ratio_end_to_end": e2e,
        "agreement": {
            "marginal_mean_diff_sd_vs_plain": diff.tolist(),
            "max_abs_mean_diff_sd_vs_plain": float(np.abs(diff).max()),
            "standard_error_sd": diff_se.tolist(),
            "plain_vs_plain_diff_sd": diff_pp.tolist(),
            "max_abs_plain_vs_plain_diff_sd": float(np.abs(diff_pp).max()),
            "plain_vs_plain_standard_error_sd": diff_pp_se.tolist(),
            "equal_length_diff_sd_vs_plain": diff_eq.tolist(),
            "max_abs_equal_length_diff_sd_vs_plain": float(np.abs(diff_eq).max()),
            "start_ensemble_diff_sd": {"plain": ((mu_plain - mu_start) / sd_ref).tolist(),
                                       "delayed_acceptance": ((mu_d - mu_start) / sd_ref).tolist()},
            "note": "delayed acceptance against the mean of the two plain runs; standard errors "
                    "sd sqrt(tau / (generations x chains)) from each run's multi-chain integrated "
                    "time; equal_length: the delayed-acceptance run's first generations (as many as "
                    "each plain run), from the same start; start_ensemble: each mean against the "
                    "mean of the common starting states"},
        "marginal_mean": {"plain": mu_b2.tolist(), "plain_replicate": mu_q.tolist(),
                          "delayed_acceptance": mu_d.tolist()},
        "marginal_sd": {"plain": sd_b2.tolist(), "delayed_acceptance": sd_d.tolist()},
        "fixed_tp": fixed_tp,
    }


def section_fixed_tp(args, model, prior, truth, cov, C, run_graph, stats, ms_ps, spectra, train, dims):
    """The same retrieval with the five T(p) parameters held at the truth (prior lo = hi):
    the posterior of the four abundances and the reference radius. Its slowest integrated
    time is tens of generations, so runs of a few thousand generations resolve it, and its
    effective sample sizes, Gelman-Rubin statistics and mean agreement are not bounded by the
    run length as the full posterior's are. After a plain burn-in, a local surrogate is
    fitted around the burned-in states as for the full posterior (this posterior's radius
    is eight times narrower than the full one's, finer than that surrogate's BF16 inputs
    resolve); then two plain batched runs and one delayed-acceptance run from the common
    burned-in state. The per-sample sampler's cost per generation is the one measured on the
    full posterior."""
    import torch
    from paper_2104_12522_amd.mcmc import Retrieval, gaussian_states
    from paper_2104_12522_amd.surrogate import MLP, Surrogate, standardisation
    d = prior.lo.size
    free = np.arange(5, d)
    lo_f, hi_f = prior.lo.copy(), prior.hi.copy()
    lo_f[:5] = hi_f[:5] = truth[:5]
    # starting states: the Laplace approximation of the free parameters given T(p)
    cond = np.linalg.inv(np.linalg.inv(cov)[np.ix_(free, free)])

    def states(n, seed):
        x = np.repeat(np.asarray(truth, np.float64)[None], n, axis=0)
        x[:, free] = gaussian_states(truth[free], cond, n, lo_f[free], hi_f[free], seed=seed)
        return torch.as_tensor(x, device="cuda")

    G, B = args.fixed_tp_gens, args.fixed_tp_burn
    G_da = 5 * G
    rb = Retrieval(model, C, lo_f, hi_f, seed=args.seed + 80, thin=10, hist_cap=B,
                   z_cap=10 * C + C * (B // 10 + 2))
    rb.resume(states(C, args.seed + 81), states(10 * C, args.seed + 82))
    t_burn = run_graph(rb, B)
    x0 = rb.s.x.clone()
    m = rb.s.archive_size
    z0 = rb.s.z[max(0, m - 10 * C):m].clone()
    hb = rb.s.history[B // 2:B].cpu().numpy().reshape(-1, d)[:, free]
    del rb
    # local surrogate: free inputs on a +-5 sd box around the burned-in states, the held
    # parameters at the truth (a unit-wide box, so that their inputs are a constant 1/2)
    t0 = time.perf_counter()
    mu_b, cov_b = hb.mean(0), np.cov(hb.T)
    sd_b = np.sqrt(np.diag(cov_b))
    lo_s, hi_s = truth - 0.5, truth + 0.5
    lo_s[free] = np.maximum(mu_b - args.surrogate_box * sd_b, prior.lo[free])
    hi_s[free] = np.minimum(mu_b + args.surrogate_box * sd_b, prior.hi[free])
    xl = np.repeat(np.asarray(truth, np.float64)[None], args.local_spectra, axis=0)
    xl[:, free] = gaussian_states(mu_b, cov_b, args.local_spectra, lo_s[free], hi_s[free],
                                  seed=args.seed + 86, inflate=2.0)
    Xl = torch.as_tensor(xl, device="cuda")
    Yl = spectra(Xl)
    mean_l, scale_l = standardisation(Yl)
    lo_t, hi_t = torch.as_tensor(lo_s, device="cuda"), torch.as_tensor(hi_s, device="cuda")
    net = MLP(dims, max_batch=5000, seed=9)
    train(net, lo_t, hi_t, Xl, Yl, mean_l, scale_l, args.epochs, 1e-3, 10)
    torch.cuda.synchronize()
    t_local = time.perf_counter() - t0
    sur = Surrogate(net, lo_t, hi_t, mean_l, scale_l, model.data, model.err, n_chains=5000)
    del Xl, Yl
    log(f"mcmc fixed T(p): burn-in {B} generations in {t_burn:.1f} s; local surrogate in "
        f"{t_local:.1f} s")

    def production(surrogate, n_gen, stream, gamma_scale=1.0):
        r = Retrieval(model, C, lo_f, hi_f, seed=args.seed + stream, thin=10, hist_cap=n_gen,
                      surrogate=surrogate, z_cap=z0.shape[0] + C * (n_gen // 10 + 1),
                      gamma_scale=gamma_scale)
        r.resume(x0, z0)
        torch.cuda.synchronize()
        wall = run_graph(r, n_gen)
        acc = r.s.n_accept.sum(0).cpu().numpy() / (C * n_gen)
        return r.s.history[:n_gen][:, :, 5:], wall, acc

    h, w, a = production(None, G, 83)
    plain, mu_1, sd_1, tau_1 = stats(h, w, a, G)
    h, w, a = production(None, G, 85)
    plain_q, mu_2, sd_2, tau_2 = stats(h, w, a, G)
    h, w, a = production(sur, G_da, 84)
    da, mu_d, sd_d, tau_d = stats(h, w, a, G_da, stage1_pass_rate=float(a[0]))
    # the same sampler with larger DE steps: the surrogate makes rejected proposals cheap, so
    # delayed acceptance can trade acceptance for step length
    gw = args.fixed_tp_da_gamma
    h, w, a = production(sur, G_da, 86, gamma_scale=gw)
    daw, mu_w, sd_w, tau_w = stats(h, w, a, G_da, stage1_pass_rate=float(a[0]), gamma_scale=gw)
    del h
    ps_wall = ms_ps * 1e-3 * G
    ps = {"ms_per_generation": ms_ps, "ess_per_s": plain["ess"] / ps_wall,
          "ess_multichain_per_s": plain["ess_multichain_min"] / ps_wall}
    sd_ref = 0.5 * (sd_1 + sd_2)
    mu_plain = 0.5 * (mu_1 + mu_2)
    se = lambda tau, n: sd_ref * np.sqrt(tau / (n * C))  # noqa: E731
    diff = (mu_d - mu_plain) / sd_ref
    diff_se = np.sqrt(0.25 * (se(tau_1, G) ** 2 + se(tau_2, G) ** 2) + se(tau_d, G_da) ** 2) / sd_ref
    diff_pp = (mu_2 - mu_1) / sd_ref
    diff_w = (mu_w - mu_plain) / sd_ref
    diff_w_se = np.sqrt(0.25 * (se(tau_1, G) ** 2 + se(tau_2, G) ** 2) + se(tau_w, G_da) ** 2) / sd_ref
    out = {"free_parameters": ["log10 x_1", "log10 x_2", "log10 x_3", "log10 x_4", "R_ref / R_J"],
           "held": {"values": truth[:5].tolist(),
                    "parameters": ["log10 kappa", "log10 gamma1", "log10 gamma2", "alpha", "beta"]},
           "burn_in": B, "local_surrogate_s": t_local, "plain_per_sample": ps, "plain_batched": plain,
           "plain_batched_replicate": plain_q, "delayed_acceptance": da,
           "ess_per_s_ratio_vs_per_sample": da["ess_per_s"] / ps["ess_per_s"],
           "ess_multichain_per_s_ratio_vs_per_sample":
               da["ess_multichain_per_s"] / ps["ess_multichain_per_s"],
           "ess_per_s_ratio_vs_batched": da["ess_per_s"] / plain["ess_per_s"],
           "ess_multichain_per_s_ratio_end_to_end":
               (da["ess_multichain_min"] / (da["wall_s"] + t_local)) / ps["ess_multichain_per_s"],
           "agreement": {"marginal_mean_diff_sd_vs_plain": diff.tolist(),
                         "max_abs_mean_diff_sd_vs_plain": float(np.abs(diff).max()),
                         "standard_error_sd": diff_se.tolist(),
                         "plain_vs_plain_diff_sd": diff_pp.tolist(),
                         "max_abs_plain_vs_plain_diff_sd": float(np.abs(diff_pp).max())},
           "delayed_acceptance_larger_steps": {
               **daw,
               "ess_per_s_ratio_vs_per_sample": daw["ess_per_s"] / ps["ess_per_s"],
               "ess_multichain_per_s_ratio_vs_per_sample":
                   daw["ess_multichain_per_s"] / ps["ess_multichain_per_s"],
               "ess_per_s_ratio_vs_batched": daw["ess_per_s"] / plain["ess_per_s"],
               "ess_multichain_per_s_ratio_end_to_end":
                   (daw["ess_multichain_min"] / (daw["wall_s"] + t_local)) / ps["ess_multichain_per_s"],
               "marginal_mean_diff_sd_vs_plain": diff_w.tolist(),
               "max_abs_mean_diff_sd_vs_plain": float(np.abs(diff_w).max()),
               "standard_error_sd": diff_w_se.tolist()},
           "marginal_mean": {"plain": mu_plain.tolist(), "delayed_acceptance": mu_d.tolist(),
                             "delayed_acceptance_larger_steps": mu_w.tolist()},
           "marginal_sd": {"plain": sd_ref.tolist(), "delayed_acceptance": sd_d.tolist(),
                           "delayed_acceptance_larger_steps": sd_w.tolist()}}
    log(f"mcmc fixed T(p): ESS plain {plain['ess']:.0f} / {plain_q['ess']:.0f} in {G} generations, "
        f"delayed acceptance {da['ess']:.0f} in {G_da}; Gelman-Rubin {plain['gelman_rubin_max']:.4f} / "
        f"{da['gelman_rubin_max']:.4f}; ESS/s vs per-sample {out['ess_per_s_ratio_vs_per_sample']:.1f}x; "
        f"max |mean diff| {np.abs(diff).max():.3f} sd (plain vs plain {np.abs(diff_pp).max():.3f} sd); "
        f"with {gw}x DE steps: ESS {daw['ess']:.0f}, Gelman-Rubin {daw['gelman_rubin_max']:.4f}, "
        f"ESS/s vs per-sample {out['delayed_acceptance_larger_steps']['ess_per_s_ratio_vs_per_sample']:.1f}x "
        f"({out['delayed_acceptance_larger_steps']['ess_multichain_per_s_ratio_vs_per_sample']:.1f}x "
        f"multi-chain), max |mean diff| {np.abs(diff_w).max():.3f} sd")
    return out


def section_mlp(args):
    """The surrogate network's kernels alone (10 -> 4 x 512 -> 1000, BF16 on the matrix cores):
    a 256-row inference and training steps at batch 512 on synthetic inputs and targets,
    timed with events; throughput against the dense BF16 peak."""
    import torch
    from paper_2104_12522_amd.surrogate import MLP, Trainer
    dims = [10, 512, 512, 512, 512, 1000]
    C, batch, n = args.chains, 512, 20480
    g = torch.Generator(device="cuda").manual_seed(args.seed + 95)
    X = torch.rand(n, dims[0], generator=g, device="cuda", dtype=torch.float64)
    Y = torch.randn(n, dims[-1], generator=g, device="cuda", dtype=torch.float64)
    lo = torch.zeros(dims[0], dtype=torch.float64, device="cuda")
    hi = torch.ones(dims[0], dtype=torch.float64, device="cuda")
    mean = torch.zeros(dims[-1], dtype=torch.float64, device="cuda")
    scale = torch.ones(dims[-1], dtype=torch.float64, device="cuda")
    net = MLP(dims, max_batch=max(C, batch), seed=11)
    out = torch.empty(C, dims[-1], dtype=torch.float32, device="cuda")
    xs = X[:C].contiguous()

    def infer():
        net.set_input(xs, lo, hi)
        net.forward(C, out)

    tr = Trainer(net, lo, hi, X, Y, mean, scale, batch=batch, seed=12)
    rows = torch.arange(batch, dtype=torch.int32, device="cuda")
    # the same network at larger training batches (throughput grows with the product sizes:
    # the batch-512 products are latency-bound)
    big = MLP(dims, max_batch=4096, seed=13)
    tr_big = {b: Trainer(big, lo, hi, X, Y, mean, scale, batch=b, seed=14) for b in (2048, 4096)}
    rows_big = {b: torch.arange(b, dtype=torch.int32, device="cuda") for b in (2048, 4096)}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    for name, fn, reps in (("inference", infer, 500), ("train_step", lambda: tr.step(rows, 1e-4), 300),
                           ("train_step_2048", lambda: tr_big[2048].step(rows_big[2048], 1e-5), 100),
                           ("train_step_4096", lambda: tr_big[4096].step(rows_big[4096], 1e-5), 100)):
        for _ in range(20):
            fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        res[name + "_us"] = e0.elapsed_time(e1) / reps * 1e3
    macs = sum(dims[i] * dims[i + 1] for i in range(len(dims) - 1))
    fl_inf = 2.0 * C * macs
    fl_step = 2.0 * batch * (3 * macs - dims[0] * dims[1])
    res.update({"dims": dims, "inference_rows": C, "train_batch": batch,
                "inference_tflops": fl_inf / (res["inference_us"] * 1e-6) / 1e12,
                "train_tflops": fl_step / (res["train_step_us"] * 1e-6) / 1e12,
                "peak_tflops": BF16_PEAK_TFLOPS})
    res["inference_frac"] = res["inference_tflops"] / BF16_PEAK_TFLOPS
    res["train_frac"] = res["train_tflops"] / BF16_PEAK_TFLOPS
    for b in (2048, 4096):
        res[f"train_tflops_{b}"] = fl_step * b / batch / (res[f"train_step_{b}_us"] * 1e-6) / 1e12
    log(f"surrogate kernels: inference {res['inference_us']:.1f} us ({res['inference_tflops']:.1f} TFLOP/s), "
        f"training step {res['train_step_us']:.1f} us ({res['train_tflops']:.1f} TFLOP/s; batch 2048 "
        f"{res['train_tflops_2048']:.1f}, 4096 {res['train_tflops_4096']:.1f} TFLOP/s)")
    return res


def section_opacity(args):
    """Line-by-line opacity build: 1e7 lines, 1e5 nu x 20 T x 100 p, float32, 25 HWHM."""
    import torch
    import workloads as wl
    import paper_2104_12522_amd as bm
    nu, temps, p_bar = wl.config4_grid()
    n_lines = args.opacity_lines
    t0 = time.time()
    lines = wl.config4_lines(n_lines)
    log(f"opacity: {n_lines} lines generated in {time.time() - t0:.1f} s")
    out = torch.empty(len(temps), len(p_bar), nu.size, dtype=torch.float32, device="cuda")
    dnu = float(nu[1] - nu[0])
    bm.opacity_table_build(lines.subset(slice(0, 1000)), temps, p_bar, float(nu[0]), dnu, nu.size,
                           out=out)
    d_lines = device_lines(lines)
    ws = bm.opacity_build_workspace(n_lines)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    bm.opacity_table_build(d_lines, temps, p_bar, float(nu[0]), dnu, nu.size, out=out, workspace=ws)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    log(f"opacity: build in {ms / 1e3:.2f} s")
    evals = window_evaluations(lines, nu, temps, p_bar, sample=20000, seed=args.seed + 80)
    res = {"lines": n_lines, "n_nu": int(nu.size), "n_temp": int(len(temps)),
           "n_p": int(len(p_bar)), "dtype": "f32 out, f64 accumulation", "cutoff_hwhm": 25.0,
           "seconds": ms / 1e3, "output_gb": out.numel() * 4 / 1e9,
           "profile_evaluations": evals, "evaluations_per_s": evals / (ms * 1e-3),
           "evaluations_note": "window points summed over lines and cells, counted on the host "
                               "from a 20000-line sample scaled to all lines"}
    del out
    res["profile_table_mode"] = table_mode_comparison(args, lines, nu, temps, p_bar)
    return res


def table_mode_comparison(args, lines, nu, temps, p_bar):
    """The paper's profile-table mode (60 x 60 Voigt profiles, oversampled and aligned to the
    output grid) against the direct build on the same subset: every 10th line, every 4th
    temperature and every 10th pressure of the grid."""
    import torch
    import paper_2104_12522_amd as bm
    sub = lines.subset(np.arange(0, lines.nu0.size, 10))
    t_sub, p_sub = temps[::4], p_bar[::10]
    dnu = float(nu[1] - nu[0])
    sn, gn = bm.VoigtTable.nodes_for(sub, t_sub, p_sub, 60, 60)
    t0 = time.perf_counter()
    tab = bm.VoigtTable(sn, gn, dnu, args.opacity_oversample, 25.0)
    torch.cuda.synchronize()
    t_table = time.perf_counter() - t0
    log(f"opacity: profile table {tab.bytes / 1e9:.2f} GB built in {t_table:.2f} s")
    shape = (len(t_sub), len(p_sub), nu.size)
    direct = torch.empty(shape, dtype=torch.float32, device="cuda")
    table = torch.empty(shape, dtype=torch.float32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    bm.opacity_table_build(sub, t_sub, p_sub, float(nu[0]), dnu, nu.size, out=direct)
    ev[1].record()
    bm.opacity_table_build_profiles(sub, t_sub, p_sub, float(nu[0]), nu.size, tab, out=table)
    ev[2].record()
    torch.cuda.synchronize()
    ms_d, ms_t = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    d = direct.double()
    big = d > 1e-3 * d.amax(dim=2, keepdim=True)
    rel = ((table.double() - d).abs() / d)[big]
    evals = window_evaluations(sub, nu, t_sub, p_sub, sample=20000, seed=args.seed + 81)
    log(f"opacity: subset direct {ms_d / 1e3:.2f} s, profile table {ms_t / 1e3:.2f} s; table vs direct "
        f"max {float(rel.max()):.2e}, median {float(rel.median()):.2e}")
    return {"lines": int(sub.nu0.size), "n_temp": int(len(t_sub)), "n_p": int(len(p_sub)),
            "profiles": "60 x 60", "oversample": args.opacity_oversample, "table_gb": tab.bytes / 1e9,
            "table_build_s": t_table, "direct_s": ms_d / 1e3, "table_mode_s": ms_t / 1e3,
            "profile_evaluations": evals, "direct_evaluations_per_s": evals / (ms_d * 1e-3),
            "table_evaluations_per_s": evals / (ms_t * 1e-3),
            "rel_diff_vs_direct_where_above_1e-3_of_max": {"max": float(rel.max()),
                                                           "median": float(rel.median()),
                                                           "p99": float(rel.quantile(0.99)) if rel.numel() < 16_000_000
                                                           else None}}


def window_evaluations(lines, nu, temps, p_bar, sample: int, seed: int) -> float:
    """Profile evaluations of a build: grid points inside each line's 25-HWHM window,
    summed over (T, p) cells, on a random sample of lines scaled to the full list."""
    k_b, amu, c_light = 1.380649e-16, 1.66053906660e-24, 2.99792458e10
    g = np.random.default_rng(seed)
    n_all = lines.nu0.size
    idx = g.choice(n_all, min(sample, n_all), replace=False)
    nu0, g296, mass = lines.nu0[idx], lines.gamma296[idx], lines.mass_amu[idx]
    dnu, n = nu[1] - nu[0], nu.size
    total = 0.0
    for t in temps:
        sig = nu0 / c_light * np.sqrt(k_b * t / (mass * amu))
        for p in p_bar:
            gam = g296 * (p / 1.01325) * np.sqrt(296.0 / t)
            hw = 25.0 * (0.5346 * gam + np.sqrt(0.2166 * gam * gam + 2.0 * np.log(2.0) * sig * sig))
            lo = np.clip(np.ceil((nu0 - hw - nu[0]) / dnu), 0, n - 1)
            hi = np.clip(np.floor((nu0 + hw - nu[0]) / dnu), -1, n - 1)
            total += float(np.maximum(hi - lo + 1, 0).sum())
    return total * n_all / idx.size


def section_copy(args):
    """A plain device copy of known size (1 GiB read + 1 GiB written), the reference that
    scales the HBM byte counters of a profiling run."""
    import torch
    n = 1 << 28
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    y.copy_(x)
    start.record()
    for _ in range(3):
        y.copy_(x)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / 3
    log(f"copy: {4 * n / 2**20:.0f} MiB in {ms:.3f} ms")
    return {"bytes_read": 4 * n, "bytes_written": 4 * n, "ms": ms,
            "gbs": 8 * n / (ms * 1e-3) / 1e9}


def cpu_model_name() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


_POOL_JOB = {}


def _oracle_spectrum(i):
    from oracle import rt as ort
    j = _POOL_JOB
    ort.forward(j["params"][i % len(j["params"])], j["setup"], j["sigma"], j["cia"])
    return i


def oracle_pool_main(path: str, budget_s: float, max_workers: int):
    """Child process of the CPU-baseline leg (no GPU in it): the FP64 oracle on spectra of
    the headline workload, first on one thread, then as a process pool over all usable
    host cores; tables memory-mapped from `path` (shared by every worker)."""
    import multiprocessing as mp
    import workloads as wl
    from oracle import rt as ort
    setup = wl.config2()
    setup.bin_width = 0
    sigma = np.load(path + "_sigma.npy", mmap_mode="r")
    cia = np.load(path + "_cia.npy")
    params = np.load(path + "_params.npy")
    # one thread
    n1, t0 = 0, time.perf_counter()
    while n1 < 3 or time.perf_counter() - t0 < min(4.0, budget_s / 4):
        ort.forward(params[n1 % len(params)], setup, sigma, cia)
        n1 += 1
    dt1 = time.perf_counter() - t0
    rate1 = n1 / dt1
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    workers = max(1, min(usable, max_workers))
    n_par = max(workers, int(rate1 * workers * budget_s * 0.8))
    _POOL_JOB.update(params=params, setup=setup, sigma=sigma, cia=cia)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        for _ in pool.imap_unordered(_oracle_spectrum, range(n_par), chunksize=1):
            pass
    dtp = time.perf_counter() - t0
    print(json.dumps({"n1": n1, "dt1": dt1, "n_par": n_par, "dtp": dtp, "workers": workers,
                      "usable": usable, "nproc": os.cpu_count(), "cpu_model": cpu_model_name()}),
          flush=True)


def cpu_baseline(sigma_np32, cia_np, params, budget_s: float, max_workers: int):
    """The FP64 oracle, as it stands, on a bounded sample of the headline workload: one
    thread, then every usable host core (a process pool over spectra), in a child process
    that never touches the GPU."""
    import subprocess
    import tempfile
    base = os.path.join("/dev/shm" if os.path.isdir("/dev/shm") else tempfile.gettempdir(),
                        f"bartmi_oracle_{os.getpid()}")
    files = [base + x for x in ("_sigma.npy", "_cia.npy", "_params.npy")]
    try:
        np.save(files[0], sigma_np32.astype(np.float64))
        np.save(files[1], cia_np)
        np.save(files[2], params)
        res = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-pool", base,
                              "--cpu-seconds", str(budget_s), "--cpu-workers", str(max_workers)],
                             capture_output=True, text=True, timeout=budget_s * 6 + 120)
    finally:
        for f in files:
            if os.path.exists(f):
                os.remove(f)
    if res.returncode != 0:
        raise RuntimeError("oracle pool failed: " + res.stderr[-2000:])
    r = json.loads(res.stdout.strip().splitlines()[-1])
    return {"value": r["n_par"] / r["dtp"], "unit": "spectra/s", "cores": r["workers"], "kind": "oracle",
            "sample": f"{r['n_par']} spectra of the full workload (100 layers x 30000 nu, 4 species), "
                      f"float64 numpy, a process pool of {r['workers']} single-threaded workers over "
                      f"spectra, {r['dtp']:.1f} s",
            "nproc": r["nproc"], "usable_cores": r["usable"], "cpu_model": r["cpu_model"],
            "single_thread": {"value": r["n1"] / r["dt1"], "spectra": r["n1"], "seconds": r["dt1"]}}


def cpu_baseline_opacity(seed: int):
    """The oracle's line-by-line build beside the library's on the same bounded sample of
    the opacity-build workload: its first 1e4 lines on its 1e5-point grid, at 1442.58 K and
    1e-8, 0.33516 and 100 bar (Doppler, intermediate and pressure-broadened cells)."""
    import torch
    import workloads as wl
    import paper_2104_12522_amd as bm
    from oracle import opacity as oop
    nu, _, _ = wl.config4_grid()
    lines = wl.config4_lines(10_000, seed=seed)
    temps, p_bar = [1442.58], [1e-8, 0.33516, 100.0]
    dnu = float(nu[1] - nu[0])
    evals = window_evaluations(lines, nu, temps, p_bar, sample=10_000, seed=seed)
    t0 = time.perf_counter()
    for p in p_bar:
        oop.cell_cross_section(lines, temps[0], p, float(nu[0]), dnu, nu.size)
    t_cpu = time.perf_counter() - t0
    out = torch.empty(1, len(p_bar), nu.size, dtype=torch.float32, device="cuda")
    d_lines = device_lines(lines)
    ws = bm.opacity_build_workspace(len(lines))
    bm.opacity_table_build(d_lines, temps, p_bar, float(nu[0]), dnu, nu.size, out=out, workspace=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    bm.opacity_table_build(d_lines, temps, p_bar, float(nu[0]), dnu, nu.size, out=out, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    t_gpu = e0.elapsed_time(e1) * 1e-3
    return {"kind": "oracle", "cores": 1, "profile_evaluations": evals,
            "oracle_s": t_cpu, "oracle_evaluations_per_s": evals / t_cpu,
            "gpu_s": t_gpu, "gpu_evaluations_per_s": evals / t_gpu,
            "sample": "first 1e4 lines of the opacity-build workload, 1e5 nu, T 1442.58 K, "
                      "p 1e-8 / 0.33516 / 100 bar; oracle float64 numpy (scipy wofz), single "
                      "thread; GPU float32 table, FP64 arithmetic"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--table", choices=("opacity", "random"), default="opacity")
    ap.add_argument("--sections", default="forward,fp64,batched,mlp,mcmc,opacity",
                    help="comma list of forward, batched, mcmc, opacity, copy")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="most processes of the CPU-baseline pool (capped by the usable cores)")
    ap.add_argument("--oracle-pool", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--seed", type=int, default=2104_12522 + 2)
    ap.add_argument("--workers", type=int, default=1,
                    help="extra multi-stream figure with W concurrent one-spectrum callers")
    ap.add_argument("--chains", type=int, default=256)
    ap.add_argument("--batched-gens", type=int, default=200)
    ap.add_argument("--no-mixed", dest="mixed", action="store_false")
    ap.add_argument("--opacity-oversample", type=int, default=1000,
                    help="fine samples per output interval of the profile table (opacity section)")
    ap.add_argument("--mcmc-gens", type=int, default=30000,
                    help="generations of each of the two plain production runs")
    ap.add_argument("--da-gens", type=int, default=150000,
                    help="generations of the delayed-acceptance production run")
    ap.add_argument("--mcmc-burn", type=int, default=1000)
    ap.add_argument("--da-burn", type=int, default=100000,
                    help="further burn-in generations with delayed acceptance before production "
                         "(two to three times the slowest integrated time of this posterior)")
    ap.add_argument("--per-sample-gens", type=int, default=200)
    ap.add_argument("--fixed-tp-gens", type=int, default=4000,
                    help="generations of each plain run on the posterior with T(p) held at the "
                         "truth (five times as many with delayed acceptance); 0 skips it")
    ap.add_argument("--fixed-tp-burn", type=int, default=2000)
    ap.add_argument("--fixed-tp-da-gamma", type=float, default=2.0,
                    help="DE step factor of the second delayed-acceptance run on the T(p)-fixed "
                         "posterior (the first uses the plain runs' factor, 1)")
    ap.add_argument("--train-spectra", type=int, default=200000)
    ap.add_argument("--surrogate-box", type=float, default=5.0,
                    help="half-width of the local surrogate's input box, in burn-in sd")
    ap.add_argument("--local-spectra", type=int, default=100000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--opacity-lines", type=int, default=10_000_000)
    ap.add_argument("--time-budget", type=float, default=540.0,
                    help="seconds the whole run may take: the sampler section shortens its two "
                         "plain production runs when its measured generation rate says they "
                         "would not fit")
    args = ap.parse_args()
    args._t0 = T_START
    if args.oracle_pool:
        oracle_pool_main(args.oracle_pool, args.cpu_seconds, args.cpu_workers)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU runs are not "
                                   "part of this build (the forward model shards by chain or "
                                   "by wavenumber range)", "n_gpus": args.gpus}))
        sys.exit(2)
    sections = [s.strip() for s in args.sections.split(",") if s.strip()]
    args._sections = sections

    import torch
    import workloads as wl

    setup = wl.config2()
    S, L, N = setup.n_species, setup.p_bar.size, setup.nu.size
    NT = len(setup.temps)
    prior = wl.line2013_prior(S)
    log(f"building tables ({args.table})")
    sigma = build_tables(setup, args.table, args.seed)
    args._sigma = sigma
    model, cia = make_model(setup, sigma, args.seed)

    out = {"metric": "forward spectra/s (100 lyr x 30k nu)", "value": None, "unit": "spectra/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": None,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "transmission forward model, 4 absorbers, 20 T x 100 layers x "
                                  "30000 nu float32 tables, H2-H2 CIA, Line-2013 T(p), 1 spectrum "
                                  "per call on one stream, 30-point bins + chi^2",
                      "table": args.table, "batch_per_call": 1, "n_layers": L, "n_nu": N,
                      "n_species": S, "n_temp": NT}}
    if "forward" in sections:
        fw = section_forward(args, setup, model, prior)
        out["value"] = fw.pop("value")
        out["ms_per_step"] = fw.pop("ms_per_step")
        out["roofline"] = fw.pop("roofline")
        out.update(fw)
    if not args.no_cpu and "forward" in sections:
        log("timing the CPU oracle")
        params_np = prior.draw(200, seed=args.seed + 1)
        out["cpu_baseline"] = cpu_baseline(sigma.cpu().numpy(), cia.cpu().numpy().astype(np.float64),
                                           params_np, args.cpu_seconds, args.cpu_workers)
        log("timing the CPU oracle's opacity build on a line subset")
        out["cpu_baseline"]["opacity_subset"] = cpu_baseline_opacity(wl.SEED_BASE + 4)
    if "fp64" in sections:
        out["fp64_single_spectrum"] = section_fp64(args)
    if "batched" in sections:
        out["batched"] = section_batched(args, setup, model, prior)
    if "mlp" in sections:
        out["surrogate_kernels"] = section_mlp(args)
    if "mcmc" in sections:
        # the retrieval labels the two visible streams (alpha <= 1/2), so that the
        # posterior has no mirror mode in (gamma1, gamma2, alpha)
        out["mcmc"] = section_mcmc(args, setup, wl.line2013_prior(S, alpha_max=0.5))
    if "copy" in sections:
        out["copy"] = section_copy(args)
    if "opacity" in sections:
        del model, sigma
        args._sigma = None
        torch.cuda.empty_cache()
        out["opacity"] = section_opacity(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
