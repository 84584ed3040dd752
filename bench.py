"""Benchmark of the transmission forward model on one MI355X.

Workload (the "full single forward model" configuration): 4 absorbers with opacity
tables on 20 temperatures (300-3000 K) x 100 log-spaced layers (1e-8--100 bar) x 30000
wavenumbers (0.5 cm^-1 from 1000 cm^-1) in float32, a 20 x 30000 H2-H2 CIA table, the
five-parameter T(p) profile, one spectrum per call. A step is one bm_forward_batch call
with B = 1: atmosphere, extinction, chord optical depth, transit depth (steps a1-a5),
and 30-point channel binning with chi^2 against a synthetic observation (a6). Every
step uses a different prior draw, so consecutive calls read different table rows.

BART runs one forward-model worker per MCMC chain, all sharing one copy of the opacity
table (Sec. 3; Sec. 4 items 8-9). The benchmark does the same: ``--workers`` concurrent
callers, each on its own HIP stream with its own workspace and outputs, each issuing
one-spectrum calls back to back (step i goes to worker i mod W). ``value`` is the
aggregate spectra/s over the timed steps; a single-stream figure is reported beside it.

Inputs are resident in HBM before timing starts. Tables come from the library's own
line-by-line opacity build (``--table opacity``, default) or from the seeded random
generator (``--table random``). One JSON line goes to stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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
        log(f"opacity table species {i}: {n_lines} lines in {time.time() - t0:.2f} s")
    return out


def cpu_baseline(setup, sigma_np, cia_np, params, budget_s: float):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload."""
    from oracle import rt as ort
    n = 0
    t0 = time.perf_counter()
    while n < len(params):
        ort.forward(params[n], setup, sigma_np, cia_np)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "spectra/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} spectra of the full workload (100 layers x 30000 nu, 4 species), "
                      f"float64 numpy, single thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--table", choices=("opacity", "random"), default="opacity")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--seed", type=int, default=2104_12522 + 2)
    ap.add_argument("--workers", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU runs are not "
                                   "part of this build (the forward model shards by chain or "
                                   "by wavenumber range, see DESIGN.md)", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import workloads as wl
    import paper_2104_12522_amd as bm

    setup = wl.config2()
    S, L, N = setup.n_species, setup.p_bar.size, setup.nu.size
    NT, NTC = len(setup.temps), len(setup.cia_temps)
    log(f"building tables ({args.table})")
    sigma = build_tables(setup, args.table, args.seed)
    cia = torch.as_tensor(wl.cia_table(setup.cia_temps, setup.nu), device="cuda")
    prior = wl.line2013_prior(S)
    n_draw = args.warmup + args.steps
    params_np = prior.draw(n_draw, seed=args.seed + 1)
    # synthetic observation: the forward model at a fixed truth plus 60 ppm noise
    truth = prior.draw(1, seed=args.seed + 2)
    nb = N // setup.bin_width
    model = bm.Model(sigma, setup.temps, setup.p_bar, setup.mass_amu, setup.tp_mode, setup.planet,
                     cia=cia, cia_temps=setup.cia_temps, bin_width=setup.bin_width,
                     data=np.zeros(nb), err=np.full(nb, 60e-6))
    f_truth = bm.Forward(model, 1, binned=True)
    f_truth(torch.as_tensor(truth, device="cuda"))
    noise = wl.rng(args.seed + 3).normal(0.0, 60e-6, nb)
    model.set_observation(f_truth.binned.cpu().numpy() + noise, np.full(nb, 60e-6))

    params = torch.as_tensor(params_np, device="cuda").contiguous()
    rows = [params[i:i + 1] for i in range(n_draw)]

    def timed(n_workers):
        streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(n_workers - 1)]
        fwds = [bm.Forward(model, 1, binned=True, chi2=True) for _ in range(n_workers)]
        for i in range(args.warmup):
            fwds[i % n_workers](rows[i], stream=streams[i % n_workers])
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        main = streams[0]
        start.record(main)
        for s_ in streams[1:]:
            s_.wait_event(start)
        t0 = time.perf_counter()
        for i in range(args.steps):
            w = i % n_workers
            fwds[w](rows[args.warmup + i], stream=streams[w])
        for s_ in streams[1:]:
            ev = torch.cuda.Event()
            ev.record(s_)
            main.wait_event(ev)
        end.record(main)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return start.elapsed_time(end) / args.steps, wall / args.steps * 1e3, int(fwds[0].flags[0])

    log(f"warmup {args.warmup}, timing {args.steps} steps on {args.workers} workers")
    ms, ms_wall, flags = timed(args.workers)
    log(f"{ms * 1e3:.2f} us per spectrum (events), {ms_wall * 1e3:.2f} us (host clock)")
    ms1 = None
    if args.workers != 1:
        ms1, _, _ = timed(1)
        log(f"single stream: {ms1 * 1e3:.2f} us per spectrum")

    # algorithmic HBM bytes of one spectrum: the two bracketing temperature rows of every
    # species table on every layer, the CIA table at most once, the spectrum and bins out
    bytes_spec = 4 * (2 * S * L * N) + 8 * NTC * N + 8 * N + 8 * nb
    achieved = bytes_spec / (ms * 1e-3) / 1e9
    out = {
        "metric": "forward spectra/s (100 lyr x 30k nu)",
        "value": 1000.0 / ms,
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "transmission forward model, 4 absorbers, 20 T x 100 layers x "
                               "30000 nu float32 tables, H2-H2 CIA, Line-2013 T(p), 1 spectrum "
                               "per call, 30-point bins + chi^2",
                   "table": args.table, "batch_per_call": 1, "workers": args.workers,
                   "n_layers": L, "n_nu": N, "n_species": S, "n_temp": NT},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": bytes_spec,
                     "timing": "HIP events around the timed loop / steps: aggregate over the "
                               "workers, atmosphere and chi^2 kernels and launch gaps included"},
        "single_stream": None if ms1 is None else {"value": 1000.0 / ms1, "ms_per_step": ms1},
        "last_flags": flags,
    }
    if not args.no_cpu:
        log("timing the CPU oracle")
        sig_np = sigma.cpu().numpy().astype(np.float64)
        cia_np = cia.cpu().numpy().astype(np.float64)
        setup_cpu = wl.config2()
        setup_cpu.bin_width = 0
        out["cpu_baseline"] = cpu_baseline(setup_cpu, sig_np, cia_np, params_np, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
