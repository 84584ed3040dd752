"""GPU parity of the forward-model steps a1-a6 against the FP64 oracle, through the C ABI.

Tolerances: FP64 mode 1e-10 relative on transit depth (1e-12 on the FP64 atmosphere);
FP32 mode 1e-4 relative on depth, and the error on the atmospheric part of the depth
(depth - r_0^2/Rs^2) is reported in ppm and held below 1e-3 of that part.
"""
import dataclasses

import numpy as np
import pytest

import workloads as wl
from oracle import atmosphere as oatm
from oracle import rt as ort

from tests._fixtures import small_config2, config1_table, gpu_model, prior_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2104_12522_amd as bm  # noqa: E402


def _np(t):
    return t.detach().cpu().numpy()


# ------------------------------------------------------------------------- a1-a2
@pytest.mark.parametrize("cfg", ["config1", "config2"])
def test_atmosphere_matches_oracle(cfg):
    if cfg == "config1":
        s, sigma = config1_table(n_nu=64)
        cia = None
        params = np.array([wl.config1_params(), [900.0, -3.0, 1.2], [1900.0, -6.5, 1.05]])
    else:
        s, sigma, cia = small_config2(n_nu=64)
        params = wl.line2013_prior(4).draw(16, seed=21)
    model = gpu_model(s, sigma, cia)
    out = bm.atmosphere(model, torch.as_tensor(params, device="cuda"))
    torch.cuda.synchronize()
    for b, th in enumerate(params):
        ref = oatm.atmosphere(th, s.p_bar, s.mass_amu, s.tp_mode, s.planet)
        np.testing.assert_allclose(_np(out["temp"][b]), ref["temp"], rtol=1e-12)
        np.testing.assert_allclose(_np(out["n_species"][b]), ref["n_species"], rtol=1e-12)
        np.testing.assert_allclose(_np(out["n_h2"][b]), ref["n_h2"], rtol=1e-12)
        np.testing.assert_allclose(_np(out["radius"][b]), ref["radius"], rtol=1e-13)
        assert int(out["flags"][b]) == ref["flags"]


# ------------------------------------------------------------------------- a3, a4, a5
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_steps_match_oracle(dtype):
    if dtype == "f64":
        s, sigma = config1_table(n_nu=1000)
        cia = None
        th = wl.config1_params()
        rt_ext, rt_tau, rt_depth = 1e-12, 1e-12, 1e-12
    else:
        s, sigma, cia = small_config2(n_nu=1000)
        th = wl.line2013_prior(4).draw(1, seed=5)[0]
        rt_ext, rt_tau, rt_depth = 1e-6, 2e-5, 1e-6
    model = gpu_model(s, sigma, cia)
    atm = oatm.atmosphere(th, s.p_bar, s.mass_amu, s.tp_mode, s.planet)
    ext_ref, fl = ort.extinction(sigma, s.temps, atm["temp"], atm["n_species"], cia, s.cia_temps,
                                 atm["n_h2"])
    ext, flags = bm.extinction(model, atm["temp"], atm["n_species"], atm["n_h2"])
    np.testing.assert_allclose(_np(ext), ext_ref, rtol=rt_ext, atol=0)
    assert int(flags[0]) == fl
    # optical depth from the oracle's extinction (rounded to the compute type)
    ext_in = torch.as_tensor(ext_ref.astype(sigma.dtype), device="cuda")
    tau = bm.optical_depth(atm["radius"], ext_in)
    tau_ref = ort.optical_depth(atm["radius"], ext_ref.astype(sigma.dtype).astype(np.float64))
    np.testing.assert_allclose(_np(tau), tau_ref, rtol=rt_tau, atol=1e-30)
    # transit depth from the oracle's optical depth
    tau_in = torch.as_tensor(tau_ref.astype(sigma.dtype), device="cuda")
    depth = bm.transit_depth(atm["radius"], tau_in, s.planet.rs_cm)
    d_ref = ort.transit_depth(atm["radius"], tau_ref.astype(sigma.dtype).astype(np.float64),
                              s.planet.rs_cm)
    np.testing.assert_allclose(_np(depth), d_ref, rtol=rt_depth)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_absorbed_fraction_accuracy(dtype):
    # two layers with r0 = 0 and Rs = r1 make the transit depth the top chord's absorbed
    # fraction 1 - exp(-tau) itself; FP32 evaluates it without expm1f (a Taylor polynomial
    # below tau = 0.35, the hardware exp2 above), claimed within 3e-7 relative everywhere
    tau1 = np.concatenate([np.logspace(-10, 2.5, 4001), np.linspace(0.34, 0.36, 2001), [0.0, 1e3]])
    tau1 = tau1.astype(np.float32 if dtype == torch.float32 else np.float64)
    tau = torch.zeros(2, tau1.size, dtype=dtype, device="cuda")
    tau[1] = torch.as_tensor(tau1, device="cuda")
    r1 = 7.0e9
    got = _np(bm.transit_depth(np.array([0.0, r1]), tau, r1))
    want = -np.expm1(-tau1.astype(np.float64))
    rtol = 3e-7 if dtype == torch.float32 else 1e-15
    m = want > 0
    print(f"{dtype}: max relative error {np.max(np.abs(got[m] - want[m]) / want[m]):.3g}")
    np.testing.assert_allclose(got, want, rtol=rtol, atol=1e-300)


def test_bin_chi2_matches_oracle():
    g = np.random.default_rng(3)
    depth = 0.02 + 1e-3 * g.random((3, 95))
    data = 0.02 + 1e-3 * g.random(9)
    err = np.full(9, 6e-5)
    binned, chi2 = bm.bin_chi2(torch.as_tensor(depth, device="cuda"), 10, data, err)
    for b in range(3):
        ref = ort.bin_spectrum(depth[b], 10)
        np.testing.assert_allclose(_np(binned[b]), ref, rtol=1e-15)
        assert float(chi2[b]) == pytest.approx(ort.chi_squared(ref, data, err), rel=1e-13)


# ------------------------------------------------------------------------- fused a1-a6
def chi2_bound(binned_ref, data, err, rtol):
    """What the channel tolerance allows chi^2 to move: each channel mean within
    rtol |b_c| of the oracle's changes its term ((b_c - d_c)/err_c)^2 by at most
    2 |r_c| e_c + e_c^2, with r_c the oracle's residual and e_c = rtol |b_c| / err_c;
    plus the double-precision rounding of the sum."""
    r = (binned_ref - data) / err
    e = rtol * np.abs(binned_ref) / err
    return float(np.sum(2.0 * np.abs(r) * e + e * e) + 1e-13 * np.sum(r * r))


def _check_fused(s, sigma, cia, params, rtol, fwd=None, data=None, err=None):
    model = gpu_model(s, sigma, cia, data=data, err=err)
    want_chi2 = data is not None
    f = bm.forward_batch(model, torch.as_tensor(params, device="cuda"),
                         binned=s.bin_width > 0, chi2=want_chi2)
    torch.cuda.synchronize()
    worst_ppm = 0.0
    for b, th in enumerate(params):
        ref = ort.forward(th, s, sigma.astype(np.float64), None if cia is None else cia.astype(np.float64),
                          data=data, err=err)
        got = _np(f.spectrum(b))
        assert int(f.flags[b]) == ref["flags"], b
        if ref["flags"] & bm.BM_FLAG_RADIUS:
            assert np.all(np.isnan(got))
            continue
        np.testing.assert_allclose(got, ref["depth"], rtol=rtol, err_msg=f"sample {b}")
        r0 = ref["atm"]["radius"][0]
        base = (r0 / s.planet.rs_cm) ** 2
        mod_err = np.max(np.abs(got - ref["depth"]))
        atm_part = np.max(ref["depth"] - base)
        worst_ppm = max(worst_ppm, 1e6 * mod_err)
        if atm_part > 0:
            assert mod_err <= 1e-3 * atm_part + 1e-15
        if s.bin_width:
            np.testing.assert_allclose(_np(f.binned_spectrum(b)), ref["binned"], rtol=rtol)
            if want_chi2:
                assert abs(float(f.chi2[b]) - ref["chi2"]) <= chi2_bound(ref["binned"], data, err, rtol)
    return worst_ppm


def test_fused_fp64_config1_parity():
    s, sigma = config1_table(n_nu=1000)
    params = np.array([wl.config1_params(), [1500.0, -3.0, 1.25], [700.0, -5.0, 1.0]])
    _check_fused(s, sigma, None, params, rtol=1e-10)


@pytest.mark.parametrize("L", [33, 100, 256])
def test_fused_fp64_many_layers(L):
    # FP64 with config-2 physics (4 absorbers, CIA, channels, chi^2): the chord weights of
    # a row block pass through 32-layer chunks, so 33 layers end a block one layer into its
    # second chunk, 100 take four, and 256 (the layer limit) take eight with the LDS
    # layout at its largest; 130 wavenumbers give two full tiles and a ragged one
    s, sigma, cia = small_config2(n_nu=130, n_layers=L, seed=140 + L)
    nb = s.nu.size // s.bin_width
    g = np.random.default_rng(141)
    data = 0.024 + 1e-4 * g.random(nb)
    err = np.full(nb, 60e-6)
    params = wl.line2013_prior(4).draw(2, seed=142 + L)
    _check_fused(s, sigma.astype(np.float64), cia, params, rtol=1e-10, data=data, err=err)


@pytest.mark.parametrize("n_nu", [1000, 1, 63, 65, 129])
def test_fused_fp32_config2_parity(n_nu):
    s, sigma, cia = small_config2(n_nu=n_nu)
    if n_nu < s.bin_width:
        s.bin_width = 0            # no complete channel: binning is rejected by the library
    params = wl.line2013_prior(4).draw(4, seed=100 + n_nu)
    ppm = _check_fused(s, sigma, cia, params, rtol=1e-4)
    print(f"n_nu={n_nu}: max |depth error| = {ppm:.3g} ppm")


def test_fused_fp32_chi2_and_bins():
    s, sigma, cia = small_config2(n_nu=995)        # 33 bins of 30 and a ragged 5-point tail
    params = wl.line2013_prior(4).draw(3, seed=7)
    nb = s.nu.size // s.bin_width
    g = np.random.default_rng(8)
    data = 0.024 + 1e-4 * g.random(nb)
    err = np.full(nb, 60e-6)
    _check_fused(s, sigma, cia, params, rtol=1e-4, data=data, err=err)


def test_fused_layers_and_flags_edge_cases():
    # two layers; temperatures outside the table; mixing ratios summing past 1
    s, sigma, cia = small_config2(n_nu=130, n_layers=2)
    s.p_bar = np.array([1.0, 0.01])
    params = np.array([
        [-1.0, -0.5, -0.2, 0.3, 1.0, -3, -4, -5, -6, 1.1],
        [0.0, 1.0, 1.0, 1.0, 1.2, -2, -2, -2, -2, 1.3],           # hot: clamps at 3000 K?
        [-1.0, -0.5, -0.2, 0.3, 1.0, -0.1, -0.2, -0.3, -0.4, 1.1],  # sum x >= 1
    ])
    _check_fused(s, sigma, cia, params, rtol=1e-4)


def test_fused_isothermal_clamp_flag():
    s, sigma = config1_table(n_nu=200)
    params = np.array([[4000.0, -4.0, 1.14], [100.0, -4.0, 1.14]])   # above / below the grid
    _check_fused(s, sigma, None, params, rtol=1e-10)


def test_fused_invalid_radius_gives_nan():
    s, sigma = config1_table(n_nu=70)
    # a huge reference radius (weak gravity there) makes 1/r negative at the top
    params = np.array([[2900.0, -4.0, 20.0], [1200.0, -4.0, 1.14]])
    _check_fused(s, sigma, None, params, rtol=1e-10)


def test_fused_mixed_instances_one_launch():
    # three models with different layer and wavenumber counts fused in one call
    setups = [small_config2(n_nu=n, n_layers=L, seed=30 + i)
              for i, (L, n) in enumerate(((60, 300), (100, 700), (150, 257)))]
    models = [gpu_model(*x) for x in setups]
    inst = [0, 1, 2, 1, 0, 2, 2]
    params = wl.line2013_prior(4).draw(len(inst), seed=41)
    f = bm.forward_batch(models, torch.as_tensor(params, device="cuda"), instance=inst, binned=True)
    torch.cuda.synchronize()
    for b, mi in enumerate(inst):
        s, sigma, cia = setups[mi]
        ref = ort.forward(params[b], s, sigma.astype(np.float64), cia.astype(np.float64))
        np.testing.assert_allclose(_np(f.spectrum(b)), ref["depth"], rtol=1e-4, err_msg=str(b))
        np.testing.assert_allclose(_np(f.binned_spectrum(b)), ref["binned"], rtol=1e-4)


def test_fused_repeat_calls_are_deterministic():
    s, sigma, cia = small_config2(n_nu=500)
    model = gpu_model(s, sigma, cia)
    params = torch.as_tensor(wl.line2013_prior(4).draw(5, seed=9), device="cuda")
    f = bm.Forward(model, 5, binned=True)
    a = f(params).depth.clone()
    ab = f.binned.clone()
    b = f(params).depth.clone()
    assert torch.equal(a, b)
    assert torch.equal(ab, f.binned)


def test_fused_full_size_sampled_against_oracle():
    """Config 2 at full size (100 layers x 30000 wavenumbers, 4 species x 20 T tables),
    in the launch configuration the benchmark times; the oracle recomputes a sample of
    wavenumber columns one by one."""
    s = wl.config2()
    sigma = wl.random_opacity_table(4, s.temps, 100, s.nu, seed=77, dtype=np.float32)
    cia = wl.cia_table(s.cia_temps, s.nu)
    model = gpu_model(s, sigma, cia)
    params = wl.line2013_prior(4).draw(2, seed=78)
    f = bm.forward_batch(model, torch.as_tensor(params, device="cuda"), binned=True)
    torch.cuda.synchronize()
    cols = np.unique(np.concatenate([[0, 1, 63, 64, 29999], np.random.default_rng(5).integers(0, 30000, 60)]))
    sub = wl.config2()
    sub.nu = s.nu[cols]
    sub.bin_width = 0
    for b in range(2):
        ref = ort.forward(params[b], sub, sigma[..., cols].astype(np.float64),
                          cia[:, cols].astype(np.float64))
        got = _np(f.spectrum(b))[cols]
        np.testing.assert_allclose(got, ref["depth"], rtol=1e-4)
        # binning is checked against the GPU's own full spectrum (property at any size)
        full = _np(f.spectrum(b))
        np.testing.assert_allclose(_np(f.binned_spectrum(b)), full.reshape(-1, 30).mean(1), rtol=1e-14)


def test_fused_channels_wider_than_a_tile():
    # 100-point channels do not fit one 64-wavenumber tile: a separate binning pass
    s, sigma, cia = small_config2(n_nu=1030)
    s.bin_width = 100
    nb = s.nu.size // s.bin_width
    g = np.random.default_rng(18)
    data = 0.024 + 1e-4 * g.random(nb)
    err = np.full(nb, 60e-6)
    params = wl.line2013_prior(4).draw(3, seed=17)
    _check_fused(s, sigma, cia, params, rtol=1e-4, data=data, err=err)


@pytest.mark.parametrize("bw", [1, 7, 64])
def test_fused_channel_widths(bw):
    s, sigma, cia = small_config2(n_nu=777)
    s.bin_width = bw
    nb = s.nu.size // bw
    data = np.full(nb, 0.025)
    err = np.full(nb, 1e-4)
    params = wl.line2013_prior(4).draw(2, seed=19 + bw)
    _check_fused(s, sigma, cia, params, rtol=1e-4, data=data, err=err)


def test_launch_configurations_match_and_tune():
    # configurations that accumulate each optical depth in the same order (all but the
    # pipelined ones, which take the layers top-down by stage) agree bit for bit; every
    # configuration matches the oracle
    s, sigma, cia = small_config2(n_nu=900, n_layers=70, seed=31)
    nb = s.nu.size // s.bin_width
    data, err = np.full(nb, 0.02), np.full(nb, 6e-5)
    model = gpu_model(s, sigma, cia, data=data, err=err)
    B = 6
    params_np = prior_for(s).draw(B, seed=32)
    params = torch.as_tensor(params_np, device="cuda")
    f = bm.Forward(model, B, binned=True, chi2=True)
    names = bm.forward_configs()
    outs = []
    for c in range(len(names)):
        f.set_config(c)
        f(params)
        outs.append((f.depth.clone(), f.binned.clone(), f.chi2.clone(), f.flags.clone()))
    groups = {}
    for c, name in enumerate(names):
        groups.setdefault("pipelined" in name, []).append(c)
    for members in groups.values():
        for c in members[1:]:
            for a, b in zip(outs[members[0]], outs[c]):
                assert torch.equal(a, b), (members[0], c)
    for c in range(len(names)):
        for b in range(B):
            ref = ort.forward(params_np[b], s, sigma.astype(np.float64), cia, data=data, err=err)
            sl = slice(int(f.depth_off[b]), int(f.depth_off[b + 1]))
            np.testing.assert_allclose(_np(outs[c][0][sl]), ref["depth"], rtol=1e-4, err_msg=str(c))
    chosen, times = f.tune(params, reps=2)
    assert 0 <= chosen < len(times) and times[chosen] > 0
    assert times[chosen] == min(t for t in times if t > 0)
    f(params)
    assert torch.equal(f.depth, outs[chosen][0]) and torch.equal(f.chi2, outs[chosen][2])
    f.set_config(-1)


def test_pipelined_configuration_layer_counts():
    # the pipelined mode covers up to 112 layers in fixed stages; check small, ragged and
    # maximal layer counts against the oracle, and its fallback above 112 layers
    names = bm.forward_configs()
    pipe = [c for c, n in enumerate(names) if "pipelined" in n]
    for L in (2, 17, 63, 112, 130):
        s, sigma, cia = small_config2(n_nu=130, n_layers=L, seed=40 + L)
        model = gpu_model(s, sigma, cia)
        params_np = prior_for(s).draw(2, seed=41)
        params = torch.as_tensor(params_np, device="cuda")
        f = bm.Forward(model, 2, binned=True)
        for c in pipe:
            f.set_config(c)
            f(params)
            torch.cuda.synchronize()
            for b in range(2):
                ref = ort.forward(params_np[b], s, sigma.astype(np.float64), cia)
                sl = slice(int(f.depth_off[b]), int(f.depth_off[b + 1]))
                np.testing.assert_allclose(_np(f.depth[sl]), ref["depth"], rtol=1e-4, err_msg=f"L={L} c={c}")
        f.set_config(-1)


def test_kernel_timing_counts_launches():
    s, sigma, cia = small_config2(n_nu=600, n_layers=60, seed=33)
    model = gpu_model(s, sigma, cia)
    f = bm.Forward(model, 2)
    params = torch.as_tensor(prior_for(s).draw(2, seed=34), device="cuda")
    with bm.KernelTiming(3) as t:
        for _ in range(5):
            f(params)
    assert t.launches == 3 and t.total_ms > 0
    with bm.KernelTiming(10) as t2:
        f(params)
    assert t2.launches == 1


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fused_optical_depth_limit(dtype):
    # Sec. 4 item 7: chords at and below the first one reaching tau_max are opaque
    if dtype == "f64":
        s, sigma = config1_table(n_nu=300)
        cia = None
        params = np.array([wl.config1_params(), [1500.0, -3.0, 1.2]])
        s.tau_max, rtol = 3.0, 1e-10
    else:
        s, sigma, cia = small_config2(n_nu=700, n_layers=80, seed=61)
        params = prior_for(s).draw(4, seed=62)
        s.tau_max, rtol = 2.0, 1e-4
    ppm = _check_fused(s, sigma, cia, params, rtol=rtol)
    # and the limit does change the spectrum
    s0 = dataclasses.replace(s, tau_max=0.0)
    model0 = gpu_model(s0, sigma, cia)
    model1 = gpu_model(s, sigma, cia)
    p = torch.as_tensor(params, device="cuda")
    d0 = bm.forward_batch(model0, p).depth.clone()
    d1 = bm.forward_batch(model1, p).depth.clone()
    assert torch.all(d1 >= d0 - 1e-15) and float((d1 - d0).max()) > 0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fused_cloud_deck_and_rayleigh(dtype):
    # Sec. 3 (gray cloud deck, H2 Rayleigh scattering) with the cloud-top pressure of the
    # Sec. 7 retrievals as the last parameter. Cases: a deck below every layer (no effect),
    # a deck above the top layer (every chord opaque: depth = (r_top / Rs)^2 exactly),
    # and decks inside the atmosphere; every launch configuration against the oracle.
    if dtype == "f64":
        s, sigma = config1_table(n_nu=300)
        cia = None
        base = np.array([wl.config1_params(), [1500.0, -3.0, 1.25], [700.0, -5.0, 1.0],
                         [1200.0, -4.0, 1.1], [1800.0, -2.5, 1.2]])
        rtol = 1e-10
    else:
        s, sigma, cia = small_config2(n_nu=700, n_layers=80, seed=71)
        base = prior_for(s).draw(5, seed=72)
        rtol = 1e-4
    s.rayleigh, s.cloud = True, True
    log_pc = np.array([3.0, -9.0, -1.3, -4.7, 0.6])
    params = np.column_stack([base, log_pc])
    assert [ort.cloud_layer(s.p_bar, v) for v in log_pc[:2]] == [-1, s.p_bar.size - 1]
    model = gpu_model(s, sigma, cia)
    assert model.n_params == params.shape[1]
    B = params.shape[0]
    f = bm.Forward(model, B)
    p = torch.as_tensor(params, device="cuda")
    refs = [ort.forward(th, s, sigma.astype(np.float64), None if cia is None else cia.astype(np.float64))
            for th in params]
    n_cfg = len(bm.forward_configs()) if dtype == "f32" else 1
    for c in range(n_cfg):
        if dtype == "f32":
            f.set_config(c)
        f(p)
        torch.cuda.synchronize()
        for b in range(B):
            sl = slice(int(f.depth_off[b]), int(f.depth_off[b + 1]))
            got = _np(f.depth[sl])
            assert int(f.flags[b]) == refs[b]["flags"]
            np.testing.assert_allclose(got, refs[b]["depth"], rtol=rtol, err_msg=f"config {c} sample {b}")
        r_top = refs[1]["atm"]["radius"][-1]
        sl = slice(int(f.depth_off[1]), int(f.depth_off[2]))
        np.testing.assert_allclose(_np(f.depth[sl]), (r_top / s.planet.rs_cm) ** 2, rtol=1e-12)
    if dtype == "f32":
        f.set_config(-1)
    # the deck and the scattering each raise the depth
    s_clear = dataclasses.replace(s, rayleigh=False, cloud=False)
    d_clear = bm.forward_batch(gpu_model(s_clear, sigma, cia),
                               torch.as_tensor(base, device="cuda")).depth.clone()
    s_ray = dataclasses.replace(s, cloud=False)
    d_ray = bm.forward_batch(gpu_model(s_ray, sigma, cia),
                             torch.as_tensor(base, device="cuda")).depth.clone()
    assert torch.all(d_ray >= d_clear) and float((d_ray - d_clear).max()) > 0
    assert torch.all(f.depth >= d_ray * (1 - 1e-6))


def test_extinction_step_rayleigh():
    # step a3 with Rayleigh scattering: the oracle's extinction plus n_H2 sigma_R(nu)
    s, sigma = config1_table(n_nu=200)
    s.rayleigh = True
    model = gpu_model(s, sigma)
    th = np.array(wl.config1_params())
    atm = oatm.atmosphere(th, s.p_bar, s.mass_amu, s.tp_mode, s.planet)
    ext_ref, _ = ort.extinction(sigma.astype(np.float64), s.temps, atm["temp"], atm["n_species"],
                                None, None, atm["n_h2"])
    ext_ref = ext_ref + atm["n_h2"][:, None] * ort.rayleigh_h2(s.nu)[None, :]
    ext, _ = bm.extinction(model, atm["temp"], atm["n_species"], atm["n_h2"])
    np.testing.assert_allclose(_np(ext), ext_ref, rtol=1e-12)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fused_h2he_cia(dtype):
    # H2-H2 and H2-He CIA (Sec. 3): the library folds the H2-He table into the H2-H2 one
    # (the filler split fixes n_He / n_H2); the oracle adds the two terms layer by layer
    s, sigma, cia = small_config2(n_nu=400, n_layers=60, seed=81)
    if dtype == "f64":
        sigma, rtol = sigma.astype(np.float64), 1e-10
    else:
        rtol = 1e-4
    cia_he = wl.cia_he_table(s.cia_temps, s.nu)
    params = prior_for(s).draw(4, seed=82)
    model = gpu_model(s, sigma, cia, cia_he=cia_he)
    f = bm.forward_batch(model, torch.as_tensor(params, device="cuda"))
    torch.cuda.synchronize()
    for b, th in enumerate(params):
        ref = ort.forward(th, s, sigma.astype(np.float64), cia.astype(np.float64), cia_he=cia_he)
        ref0 = ort.forward(th, s, sigma.astype(np.float64), cia.astype(np.float64))
        assert int(f.flags[b]) == ref["flags"]
        np.testing.assert_allclose(_np(f.spectrum(b)), ref["depth"], rtol=rtol, err_msg=f"sample {b}")
        assert np.max(ref["depth"] - ref0["depth"]) > 0      # the H2-He term is visible


def test_cia_combine_entry_point():
    g = np.random.default_rng(9)
    a, b = g.uniform(1e-48, 1e-45, 1000), g.uniform(1e-48, 1e-45, 1000)
    ta, tb = torch.as_tensor(a, device="cuda"), torch.as_tensor(b, device="cuda")
    out = torch.empty_like(ta)
    lib = bm.lib()
    assert lib.bm_cia_combine(bm._ptr(ta), bm._ptr(tb), 0.15 / 0.85, 1000, bm._ptr(out), bm._stream()) == 0
    torch.cuda.synchronize()
    np.testing.assert_allclose(_np(out), a + (0.15 / 0.85) * b, rtol=1e-15)
    assert lib.bm_cia_combine(bm._ptr(ta), bm._ptr(tb), float("nan"), 1000, bm._ptr(out), bm._stream()) != 0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_emission_geometry_matches_oracle(dtype):
    # eclipse geometry (emergent intensity, Planck source, vertical optical depth) through
    # bm_forward_batch, with channels and chi^2 from the separate binning pass
    s, sigma, cia = small_config2(n_nu=700, n_layers=70, seed=91)
    s.geometry = "eclipse"
    if dtype == "f64":
        sigma, rtol = sigma.astype(np.float64), 1e-10
    else:
        rtol = 1e-4
    params = prior_for(s).draw(4, seed=92)
    ref0 = ort.forward(params[0], s, sigma.astype(np.float64), cia.astype(np.float64))
    nb = s.nu.size // s.bin_width
    data = ref0["binned"] * (1.0 + 1e-3 * np.sin(np.arange(nb)))
    err = 1e-3 * ref0["binned"]
    _check_fused(s, sigma, cia, params, rtol=rtol, data=data, err=err)


def test_emission_isothermal_is_a_blackbody():
    # f08isothermal (Sec. 6): an isothermal atmosphere emits the Planck function
    s, sigma = config1_table(n_nu=300)
    s.geometry = "eclipse"
    model = gpu_model(s, sigma)
    params = np.array([[1200.0, -4.0, 1.14], [2100.0, -3.0, 1.2]])
    f = bm.forward_batch(model, torch.as_tensor(params, device="cuda"))
    torch.cuda.synchronize()
    for b in range(2):
        np.testing.assert_allclose(_np(f.spectrum(b)), ort.planck(s.nu, params[b, 0]), rtol=1e-12)


def test_emission_rejects_transit_only_options():
    s, sigma = config1_table(n_nu=64)
    s.geometry, s.tau_max = "eclipse", 2.0
    model = gpu_model(s, sigma)
    with pytest.raises(bm.BartmiError):
        bm.forward_batch(model, torch.as_tensor(np.array([[1200.0, -4.0, 1.14]]), device="cuda"))


# ------------------------------------------------------------------------- tile-major tables
@pytest.mark.parametrize("n_nu,tw", [(130, 60), (130, 64), (129, 7), (61, 1), (995, 60)])
def test_sigma_tiles_copy_is_exact(n_nu, tw):
    # out[s][k][t][l][c] = sigma[s][k][l][min(t tw + c, Nnu - 1)], c < tw, element for element
    s, sigma, cia = small_config2(n_nu=n_nu, n_layers=17, seed=50)
    model = gpu_model(s, sigma, cia, tiles=False)
    model.build_tiles(tw)
    torch.cuda.synchronize()
    S, NT, L, N = sigma.shape
    n_tiles = -(-N // tw)
    nu = np.minimum(np.arange(n_tiles)[:, None] * tw + np.arange(tw)[None, :], N - 1)   # [t][c]
    want = sigma[:, :, :, nu].transpose(0, 1, 3, 2, 4)                                  # [s][k][t][l][c]
    got = _np(model.sigma_tiles).reshape(S, NT, n_tiles, L, tw)
    assert np.array_equal(got, want)
    assert model.struct.tile_w == tw


def _all_configs(model, params, binned, chi2):
    f = bm.Forward(model, params.shape[0], binned=binned, chi2=chi2)
    outs = []
    for c in range(len(bm.forward_configs())):
        f.set_config(c)
        f(params)
        outs.append([t.clone() for t in (f.depth, f.binned, f.chi2, f.flags) if t is not None])
    f.set_config(-1)
    torch.cuda.synchronize()
    return outs


@pytest.mark.parametrize("n_nu,L,B", [(995, 100, 1), (995, 100, 3), (900, 70, 2), (130, 130, 2), (61, 17, 1)])
def test_tiled_tables_give_identical_results(n_nu, L, B):
    # the tile-major copy holds the same values, so every launch configuration gives the
    # same depth, channels, chi^2 and flags bit for bit with and without it (binned calls
    # use the copy; unbinned calls have tile width 64 and read the row-major tables)
    s, sigma, cia = small_config2(n_nu=n_nu, n_layers=L, seed=60 + L)
    nb = s.nu.size // s.bin_width
    data, err = np.full(nb, 0.02), np.full(nb, 6e-5)
    params = torch.as_tensor(prior_for(s).draw(B, seed=61), device="cuda")
    plain = gpu_model(s, sigma, cia, data=data, err=err, tiles=False)
    tiled = gpu_model(s, sigma, cia, data=data, err=err)
    assert tiled.sigma_tiles is not None and tiled.struct.tile_w == 60
    for binned in (True, False):
        a = _all_configs(plain, params, binned, binned)
        b = _all_configs(tiled, params, binned, binned)
        for c, (x, y) in enumerate(zip(a, b)):
            for u, v in zip(x, y):
                assert torch.equal(u, v), (binned, c)
    # and against the oracle (binned call, default configuration)
    f = bm.Forward(tiled, B, binned=True, chi2=True)
    f(params)
    for b_ in range(B):
        ref = ort.forward(_np(params[b_]), s, sigma.astype(np.float64), cia, data=data, err=err)
        sl = slice(int(f.depth_off[b_]), int(f.depth_off[b_ + 1]))
        np.testing.assert_allclose(_np(f.depth[sl]), ref["depth"], rtol=1e-4)


def test_tiled_tables_fp64_and_mixed_instances():
    # FP64 (config 1 shapes, no channels: tile width 64) and a mixed batch of two
    # instances, each with its own copy, against the row-major tables
    s, sigma = config1_table(n_nu=1000)
    params = torch.as_tensor(np.array([wl.config1_params(), [1500.0, -3.0, 1.25]]), device="cuda")
    outs = []
    for tiles in (False, True):
        model = gpu_model(s, sigma, None, tiles=tiles)
        f = bm.forward_batch(model, params, binned=False, chi2=False)
        torch.cuda.synchronize()
        outs.append(f.depth.clone())
    assert torch.equal(outs[0], outs[1])
    inst = [(60, 800), (100, 995)]
    setups = [small_config2(n_nu=n, n_layers=L, seed=70 + L) for L, n in inst]
    params_np = wl.line2013_prior(4).draw(4, seed=71)
    res = []
    for tiles in (False, True):
        models = [gpu_model(st, sg, ci, tiles=tiles) for st, sg, ci in setups]
        f = bm.Forward(models, 4, instance=[0, 1, 1, 0], binned=True)
        f(torch.as_tensor(params_np, device="cuda"))
        torch.cuda.synchronize()
        res.append((f.depth.clone(), f.binned.clone()))
    assert torch.equal(res[0][0], res[1][0]) and torch.equal(res[0][1], res[1][1])


@pytest.mark.parametrize("n_on", [0, 1, 3, 4, 5, 9, 16, 17, 40])
def test_masked_calls_match_unmasked(n_on):
    # a masked call of one run of samples prepares records and launches the forward kernel
    # over the list of requested samples only, in a few slots that take the list's entries
    # in turn (16 per tile, 4 with pipelined stages; more requested samples than slots make
    # slots take several): requested samples get exactly the unmasked call's depth,
    # channels, chi^2 and flags in every configuration, the others' outputs are left as
    # they were
    s, sigma, cia = small_config2(n_nu=995, n_layers=70, seed=90)
    nb = s.nu.size // s.bin_width
    data, err = np.full(nb, 0.02), np.full(nb, 6e-5)
    model = gpu_model(s, sigma, cia, data=data, err=err)
    B = 40
    params = torch.as_tensor(prior_for(s).draw(B, seed=91), device="cuda")
    on = np.zeros(B, dtype=np.int32)
    on[np.random.default_rng(92).choice(B, n_on, replace=False)] = 1
    act = torch.as_tensor(on, device="cuda")
    f = bm.Forward(model, B, binned=True, chi2=True)
    for c in range(len(bm.forward_configs())):
        f.set_config(c)
        f(params)
        ref = [t.clone() for t in (f.depth, f.binned, f.chi2, f.flags)]
        for t in (f.depth, f.binned, f.chi2):
            t.fill_(-7.0)
        f.flags.fill_(-7)
        f(params, active=act)
        torch.cuda.synchronize()
        for b in range(B):
            d = slice(int(f.depth_off[b]), int(f.depth_off[b + 1]))
            k = slice(int(f.bin_off[b]), int(f.bin_off[b + 1]))
            if on[b]:
                assert torch.equal(f.depth[d], ref[0][d]) and torch.equal(f.binned[k], ref[1][k]), (c, b)
                assert torch.equal(f.chi2[b], ref[2][b]) and int(f.flags[b]) == int(ref[3][b]), (c, b)
            else:
                assert bool((f.depth[d] == -7.0).all()) and bool((f.binned[k] == -7.0).all()), (c, b)
                assert float(f.chi2[b]) == -7.0 and int(f.flags[b]) == -7, (c, b)
    f.set_config(-1)


def test_masked_calls_beyond_the_pipelined_layers():
    # 150 layers (more than the pipelined and staged modes hold): a masked call with the
    # batch pinned to streamed chord weights matches the unmasked call
    s, sigma, cia = small_config2(n_nu=300, n_layers=150, seed=93)
    nb = s.nu.size // s.bin_width
    model = gpu_model(s, sigma, cia, data=np.full(nb, 0.02), err=np.full(nb, 6e-5))
    B = 20
    params = torch.as_tensor(prior_for(s).draw(B, seed=94), device="cuda")
    on = np.zeros(B, dtype=np.int32)
    on[[2, 7, 19]] = 1
    act = torch.as_tensor(on, device="cuda")
    f = bm.Forward(model, B, binned=True, chi2=True)
    names = bm.forward_configs()
    streamed = [c for c, n in enumerate(names) if "streamed" in n and n.startswith("cached")][0]
    f.set_config(streamed)
    f(params)
    ref = [t.clone() for t in (f.depth, f.chi2)]
    f.depth.fill_(-7.0)
    f(params, active=act)
    torch.cuda.synchronize()
    for b in range(B):
        d = slice(int(f.depth_off[b]), int(f.depth_off[b + 1]))
        if on[b]:
            assert torch.equal(f.depth[d], ref[0][d]) and torch.equal(f.chi2[b], ref[1][b]), b
        else:
            assert bool((f.depth[d] == -7.0).all()), b
    f.set_config(-1)


@pytest.mark.parametrize("B", [1024, 1100])
def test_masked_calls_on_both_sides_of_the_preparation_built_list(B):
    # up to 1024 samples the record preparation builds the list of requested samples
    # itself; beyond, a list kernel runs first: both give the unmasked call's results for the
    # requested samples (first, last and scattered ones) and leave the others untouched
    s, sigma, cia = small_config2(n_nu=120, n_layers=60, seed=95)
    nb = s.nu.size // s.bin_width
    model = gpu_model(s, sigma, cia, data=np.full(nb, 0.02), err=np.full(nb, 6e-5))
    params = torch.as_tensor(prior_for(s).draw(B, seed=96), device="cuda")
    on = np.zeros(B, dtype=np.int32)
    on[[0, 5, 511, 512, 777, B - 2, B - 1]] = 1
    act = torch.as_tensor(on, device="cuda")
    f = bm.Forward(model, B, binned=True, chi2=True)
    f(params)
    ref = [t.clone() for t in (f.depth, f.chi2, f.flags)]
    f.depth.fill_(-7.0)
    f.chi2.fill_(-7.0)
    f(params, active=act)
    torch.cuda.synchronize()
    for b in range(B):
        d = slice(int(f.depth_off[b]), int(f.depth_off[b + 1]))
        if on[b]:
            assert torch.equal(f.depth[d], ref[0][d]) and torch.equal(f.chi2[b], ref[1][b]), b
        else:
            assert bool((f.depth[d] == -7.0).all()) and float(f.chi2[b]) == -7.0, b
