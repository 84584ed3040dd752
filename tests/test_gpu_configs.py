"""Parity at the workloads' own shapes, through the C ABI, against the oracle:

- the FP64 single-spectrum workload end to end (one absorber, 1e4 lines): the library's
  line-by-line table build, then the FP64 forward model on that table, against the
  oracle's brute-force table and forward model (depth at 1e-10 relative);
- the mixed batch at full size (60 layers x 8000, 100 x 30000 and 150 x 50000
  wavenumbers, each instance with its own 20-temperature tables) in one launch, in the
  autotuned configuration that the benchmark times; the oracle computes every spectrum
  whole (depth at 1e-4 relative, channels, chi^2 within the bound the channel tolerance
  implies).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import opacity as oop
from oracle import rt as ort

from tests._fixtures import gpu_model
from tests.test_gpu_forward import chi2_bound

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2104_12522_amd as bm  # noqa: E402


def _np(t):
    return t.detach().cpu().numpy()


def test_fp64_single_spectrum_workload_end_to_end():
    s = wl.config1()
    lines = wl.line_list(s.lines_per_species[0], seed=wl.SEED_BASE + 1, mass_amu=float(s.mass_amu[0]))
    dnu = float(s.nu[1] - s.nu[0])
    print(f"[case] config-1 table build: {len(lines)} lines, {s.temps.size} T x {s.p_bar.size} p x "
          f"{s.nu.size} nu", flush=True)
    table = bm.opacity_table_build(lines, s.temps, s.p_bar, float(s.nu[0]), dnu, s.nu.size, dtype=torch.float64)
    torch.cuda.synchronize()
    ref_table = oop.opacity_table(lines, s.temps, s.p_bar, float(s.nu[0]), dnu, s.nu.size)
    got_table = _np(table)
    scale = ref_table.max()
    np.testing.assert_allclose(got_table, ref_table, rtol=1e-9, atol=1e-13 * scale)
    sigma_gpu = table.reshape(1, *table.shape).contiguous()
    model = bm.Model(sigma_gpu, s.temps, s.p_bar, s.mass_amu, s.tp_mode, s.planet, device="cuda")
    params = np.array([wl.config1_params(), [900.0, -3.0, 1.2], [2500.0, -5.5, 1.05]])
    f = bm.forward_batch(model, torch.as_tensor(params, device="cuda"))
    torch.cuda.synchronize()
    for b, th in enumerate(params):
        ref = ort.forward(th, s, ref_table[None], None)
        got = _np(f.spectrum(b))
        assert int(f.flags[b]) == ref["flags"]
        np.testing.assert_allclose(got, ref["depth"], rtol=1e-10, err_msg=f"sample {b}")
        # the absorber changes the depth: the comparison is not of the opaque disk alone
        r0 = ref["atm"]["radius"][0]
        assert np.max(ref["depth"]) - (r0 / s.planet.rs_cm) ** 2 > 1e-4 * np.max(ref["depth"])


def test_mixed_batch_full_size():
    setups = wl.config3_mixed()
    sigmas, cias, models = [], [], []
    for k, s in enumerate(setups):
        print(f"[case] mixed batch instance {k}: {s.p_bar.size} layers x {s.nu.size} nu", flush=True)
        sig = wl.random_opacity_table(4, s.temps, s.p_bar.size, s.nu, seed=300 + k, dtype=np.float32)
        cia = wl.cia_table(s.cia_temps, s.nu)
        nb = s.nu.size // s.bin_width
        g = np.random.default_rng(310 + k)
        data = 0.021 + 2e-4 * g.random(nb)
        err = np.full(nb, 60e-6)
        models.append(gpu_model(s, sig, cia, data=data, err=err))
        sigmas.append(sig.astype(np.float64))
        cias.append((cia.astype(np.float64), data, err))
        del sig
    inst = [0, 1, 2, 2, 1, 0, 2, 1]
    params = wl.line2013_prior(4).draw(len(inst), seed=320)
    p_dev = torch.as_tensor(params, device="cuda")
    f = bm.Forward(models, len(inst), instance=inst, binned=True, chi2=True)
    chosen, _ = f.tune(p_dev, reps=2)
    print(f"[case] mixed batch: tuned configuration {chosen}", flush=True)
    f(p_dev)
    torch.cuda.synchronize()
    for b, mi in enumerate(inst):
        s = setups[mi]
        cia, data, err = cias[mi]
        ref = ort.forward(params[b], s, sigmas[mi], cia, data=data, err=err)
        assert int(f.flags[b]) == ref["flags"], b
        np.testing.assert_allclose(_np(f.spectrum(b)), ref["depth"], rtol=1e-4, err_msg=f"sample {b}")
        np.testing.assert_allclose(_np(f.binned_spectrum(b)), ref["binned"], rtol=1e-4)
        assert abs(float(f.chi2[b]) - ref["chi2"]) <= chi2_bound(ref["binned"], data, err, 1e-4)
