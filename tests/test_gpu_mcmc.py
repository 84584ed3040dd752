"""GPU DE-MCz sampler against the reference sampler (same counter-based random stream),
statistical checks on a known target, and graph capture of whole generations."""
import numpy as np
import pytest

import workloads as wl
from oracle import mcmc as om
from oracle import rt as ort

from tests._fixtures import small_config2, gpu_model

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2104_12522_amd as bm  # noqa: E402
from paper_2104_12522_amd.mcmc import DEMCz, Retrieval  # noqa: E402


def _np(t):
    return t.detach().cpu().numpy()


PRIOR = wl.line2013_prior(4)


@pytest.mark.parametrize("p_snooker,gscale", [(0.0, 1.0), (0.5, 1.0), (0.0, 0.3)])
def test_init_and_proposals_match_reference(p_snooker, gscale):
    C, seed, z_init = 37, 987654321, 100
    s = DEMCz(C, PRIOR.lo, PRIOR.hi, seed, z_cap=400, p_snooker=p_snooker, gamma_scale=gscale)
    s.init(z_init)
    x_ref, z_ref = om.init_state(seed, C, z_init, PRIOR.lo, PRIOR.hi)
    torch.cuda.synchronize()
    assert np.array_equal(_np(s.x), x_ref)
    assert np.array_equal(_np(s.z)[:z_init], z_ref)
    assert s.archive_size == z_init and s.generation == 0
    s.propose()
    y_ref, lq_ref = om.propose_zs(x_ref, z_ref, z_init, 0, seed, PRIOR.lo, PRIOR.hi, 1e-6, p_snooker, gscale)
    # DE moves carry normals (device log/cos); snooker moves are +-*/ only: bit-exact
    np.testing.assert_allclose(_np(s.prop), y_ref, rtol=4.5e-16, atol=1e-300)
    snk = lq_ref != 0.0
    assert np.array_equal(_np(s.prop)[snk], y_ref[snk])
    np.testing.assert_allclose(_np(s.log_q), lq_ref, rtol=1e-13, atol=1e-15)
    if p_snooker > 0:
        assert 5 < snk.sum() < C - 5


def test_fixed_parameters_match_reference():
    # log gamma1 and alpha held at -0.6 and 0.3 (zero-width prior): gamma and the snooker
    # factor count the eight free parameters, and no move changes the fixed two
    lo, hi = PRIOR.lo.copy(), PRIOR.hi.copy()
    lo[[1, 3]] = hi[[1, 3]] = [-0.6, 0.3]
    C, seed, z_init = 37, 13579, 100
    s = DEMCz(C, lo, hi, seed, z_cap=400, p_snooker=0.5)
    assert s.struct.n_free == 8
    s.init(z_init)
    x_ref, z_ref = om.init_state(seed, C, z_init, lo, hi)
    torch.cuda.synchronize()
    assert np.array_equal(_np(s.x), x_ref) and np.all(x_ref[:, [1, 3]] == [-0.6, 0.3])
    assert np.array_equal(_np(s.z)[:z_init], z_ref)
    s.propose()
    y_ref, lq_ref = om.propose_zs(x_ref, z_ref, z_init, 0, seed, lo, hi, 1e-6, 0.5)
    y = _np(s.prop)
    assert np.all(y[:, [1, 3]] == [-0.6, 0.3])
    np.testing.assert_allclose(y, y_ref, rtol=4.5e-16, atol=1e-300)
    snk = lq_ref != 0.0
    assert 5 < snk.sum() < C - 5 and np.array_equal(y[snk], y_ref[snk])
    np.testing.assert_allclose(_np(s.log_q), lq_ref, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("p_snooker", [0.0, 0.5])
def test_accept_bookkeeping_matches_reference(p_snooker):
    C, seed, d = 64, 4242, PRIOR.lo.size
    s = DEMCz(C, PRIOR.lo, PRIOR.hi, seed, thin=3, z_cap=1000, hist_cap=8, p_snooker=p_snooker)
    s.init(50)
    g = np.random.default_rng(1)
    chi2_x = g.uniform(50, 100, C)
    s.set_lp(torch.as_tensor(chi2_x, device="cuda"))
    x = _np(s.x).copy()
    z = _np(s.z)[:50].copy()
    lp = -0.5 * chi2_x
    for gen in range(7):
        s.propose()
        y = _np(s.prop)
        chi2_y = g.uniform(45, 105, C)
        flags = (g.random(C) < 0.05).astype(np.int32)
        s.accept(torch.as_tensor(chi2_y, device="cuda"), torch.as_tensor(flags, device="cuda"))
        y_ref, lq_ref = om.propose_zs(x, z, len(z), gen, seed, PRIOR.lo, PRIOR.hi, 1e-6, p_snooker)
        np.testing.assert_allclose(y, y_ref, rtol=4.5e-16, atol=1e-300)
        lq = _np(s.log_q).copy()
        np.testing.assert_allclose(lq, lq_ref, rtol=1e-13, atol=1e-15)
        x, lp, taken = om.accept(x, lp, y, chi2_y, flags, gen, seed, PRIOR.lo, PRIOR.hi, lq)
        if (gen + 1) % 3 == 0:
            z = np.vstack([z, x])
        torch.cuda.synchronize()
        assert np.array_equal(_np(s.x), x)
        np.testing.assert_array_equal(_np(s.lp), lp)
        np.testing.assert_array_equal(_np(s.history)[gen], x)
    assert s.generation == 7 and s.archive_size == len(z)
    np.testing.assert_array_equal(_np(s.z)[:len(z)], z)


@pytest.mark.parametrize("p_snooker", [0.0, 0.5])
def test_delayed_acceptance_steps_match_reference(p_snooker):
    C, seed = 48, 77
    s = DEMCz(C, PRIOR.lo, PRIOR.hi, seed, thin=10, z_cap=500, surrogate=True, p_snooker=p_snooker)
    s.init(60)
    g = np.random.default_rng(2)
    chi2_x, chi2s_x = g.uniform(50, 100, C), g.uniform(50, 100, C)
    s.set_lp(torch.as_tensor(chi2_x, device="cuda"), None, torch.as_tensor(chi2s_x, device="cuda"))
    x, z = _np(s.x).copy(), _np(s.z)[:60].copy()
    lp, ls = -0.5 * chi2_x, -0.5 * chi2s_x
    active = torch.zeros(C, dtype=torch.int32, device="cuda")
    for gen in range(5):
        s.propose()
        y = _np(s.prop)
        cs = g.uniform(45, 105, C)
        s.da_screen(torch.as_tensor(cs, device="cuda"), active)
        lq = _np(s.log_q).copy()
        if p_snooker > 0:
            _, lq_ref = om.propose_zs(x, z, len(z), gen, seed, PRIOR.lo, PRIOR.hi, 1e-6, p_snooker)
            np.testing.assert_allclose(lq, lq_ref, rtol=1e-13, atol=1e-15)
        act_ref = om.da_screen(y, cs, ls, gen, seed, PRIOR.lo, PRIOR.hi, lq)
        torch.cuda.synchronize()
        assert np.array_equal(_np(active), act_ref)
        ce = g.uniform(45, 105, C)
        s.da_accept(torch.as_tensor(ce, device="cuda"), None, torch.as_tensor(cs, device="cuda"), active)
        x, lp, ls = om.da_accept(x, lp, ls, y, ce, None, cs, act_ref, gen, seed, PRIOR.lo, PRIOR.hi)
        torch.cuda.synchronize()
        assert np.array_equal(_np(s.x), x)
        np.testing.assert_array_equal(_np(s.lp), lp)
        np.testing.assert_array_equal(_np(s.lp_surr), ls)


@pytest.mark.parametrize("p_snooker", [0.0, 0.1, 1.0])
def test_gaussian_target_on_gpu(p_snooker):
    mu = torch.tensor([0.3, -0.2, 0.5], dtype=torch.float64, device="cuda")
    sd = torch.tensor([0.2, 0.1, 0.3], dtype=torch.float64, device="cuda")
    lo, hi = np.full(3, -3.0), np.full(3, 3.0)
    C, n_gen = 64, 1500
    s = DEMCz(C, lo, hi, 5, thin=5, z_cap=30 + C * n_gen // 5 + C, hist_cap=n_gen, p_snooker=p_snooker)

    def chi2(y):
        return (((y - mu) / sd) ** 2).sum(1).contiguous()
    s.init(30)
    s.set_lp(chi2(s.x))
    for _ in range(n_gen):
        s.propose()
        s.accept(chi2(s.prop))
    h = _np(s.history)[300:].reshape(-1, 3)
    n_eff = h.shape[0] / 20
    se = _np(sd) / np.sqrt(n_eff)
    assert np.all(np.abs(h.mean(0) - _np(mu)) < 5 * se)
    np.testing.assert_allclose(h.std(0), _np(sd), rtol=0.1)


def _retrieval_setup(n_chains=32):
    s, sigma, cia = small_config2(n_nu=600, n_layers=60, seed=51)
    truth = np.array([-1.5, -0.6, 0.2, 0.3, 0.9, -3.5, -4.0, -5.0, -6.0, 1.15])
    ref = ort.forward(truth, s, sigma.astype(np.float64), cia)
    nb = s.nu.size // s.bin_width
    err = np.full(nb, 60e-6)
    data = ref["binned"] + wl.rng(3).normal(0, 60e-6, nb)
    model = gpu_model(s, sigma, cia, data=data, err=err)
    return model, truth


def test_retrieval_graph_replay_matches_eager():
    model, _ = _retrieval_setup()
    eager = Retrieval(model, 32, PRIOR.lo, PRIOR.hi, seed=123, thin=2, hist_cap=16)
    eager.start()
    eager.run(12)
    torch.cuda.synchronize()
    graphed = Retrieval(model, 32, PRIOR.lo, PRIOR.hi, seed=123, thin=2, hist_cap=16)
    graphed.start()
    g = graphed.capture(4)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()             # eager host work between replays
        _ = float(graphed.s.lp.sum())
    assert graphed.s.generation == 12
    assert torch.equal(eager.s.x, graphed.s.x)
    assert torch.equal(eager.s.lp, graphed.s.lp)
    assert torch.equal(eager.s.history, graphed.s.history)
    assert torch.equal(eager.s.z, graphed.s.z)


def test_retrieval_with_fixed_parameters():
    # the five T(p) parameters held at the truth (lo = hi): every state of a graph-captured
    # run with snooker moves keeps them, the others move, and the sampler counts five free
    # parameters
    model, truth = _retrieval_setup()
    lo, hi = PRIOR.lo.copy(), PRIOR.hi.copy()
    lo[:5] = hi[:5] = truth[:5]
    r = Retrieval(model, 32, lo, hi, seed=77, thin=2, hist_cap=20)
    assert r.s.struct.n_free == 5
    r.start()
    g = r.capture(10)
    g.replay()
    g.replay()
    torch.cuda.synchronize()
    h = _np(r.s.history)
    assert np.all(h[:, :, :5] == truth[:5])
    assert np.all(_np(r.s.z)[:r.s.archive_size, :5] == truth[:5])
    assert int(r.s.n_accept[:, 1].sum()) > 0
    assert np.all(h[-1, :, 5:].std(axis=0) > 0)


def test_retrieval_chi2_matches_oracle_for_accepted_states():
    model, _ = _retrieval_setup()
    r = Retrieval(model, 32, PRIOR.lo, PRIOR.hi, seed=9, thin=2)
    r.start()
    r.run(6)
    torch.cuda.synchronize()
    s, sigma, cia = small_config2(n_nu=600, n_layers=60, seed=51)
    data, err = model.data.cpu().numpy(), model.err.cpu().numpy()
    x, lp = _np(r.s.x), _np(r.s.lp)
    checked = 0
    for c in range(32):
        ref = ort.forward(x[c], s, sigma.astype(np.float64), cia, data=data, err=err)
        if not np.isfinite(lp[c]):
            assert ref["flags"] != 0          # flagged models have zero posterior
            continue
        assert -2 * lp[c] == pytest.approx(ref["chi2"], rel=1e-3)
        checked += 1
    assert checked > 10


def test_masked_forward_leaves_inactive_samples_untouched():
    model, _ = _retrieval_setup()
    f = bm.Forward(model, 8, binned=True, chi2=True)
    p = torch.as_tensor(PRIOR.draw(8, seed=4), device="cuda")
    f(p)
    d0, c0 = f.depth.clone(), f.chi2.clone()
    active = torch.tensor([1, 0, 1, 0, 0, 1, 0, 1], dtype=torch.int32, device="cuda")
    p2 = torch.as_tensor(PRIOR.draw(8, seed=5), device="cuda")
    f(p2, active=active)
    full = bm.Forward(model, 8, binned=True, chi2=True)
    full(p2)
    torch.cuda.synchronize()
    for b in range(8):
        sl = slice(int(f.depth_off[b]), int(f.depth_off[b + 1]))
        if active[b]:
            assert torch.equal(f.depth[sl], full.depth[sl]) and f.chi2[b] == full.chi2[b]
        else:
            assert torch.equal(f.depth[sl], d0[sl]) and f.chi2[b] == c0[b]


def test_surrogate_stage_cuts_exact_evaluations():
    """What the learned surrogate gains: as stage 1 of delayed acceptance it spares most
    exact forward evaluations while the exact model, as stage 2, keeps the acceptances."""
    import math
    from paper_2104_12522_amd.mcmc import fisher_covariance, gaussian_states
    from paper_2104_12522_amd.surrogate import MLP, Surrogate, Trainer, standardisation
    model, truth = _retrieval_setup()
    C, burn, n_gen = 64, 300, 400
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")  # noqa: E731
    cov = fisher_covariance(model, truth, PRIOR.lo, PRIOR.hi)
    rb = Retrieval(model, C, PRIOR.lo, PRIOR.hi, seed=21, thin=5, hist_cap=burn,
                   z_cap=8 * C + C * (burn // 5 + 2))
    rb.resume(dev(gaussian_states(truth, cov, C, PRIOR.lo, PRIOR.hi, seed=22)),
              dev(gaussian_states(truth, cov, 8 * C, PRIOR.lo, PRIOR.hi, seed=23)))
    rb.run(burn)
    hb = rb.s.history[burn // 2:burn].cpu().numpy().reshape(-1, PRIOR.lo.size)
    mu, cb = hb.mean(0), np.cov(hb.T)
    sd = np.sqrt(np.diag(cb))
    lo, hi = np.maximum(mu - 5 * sd, PRIOR.lo), np.minimum(mu + 5 * sd, PRIOR.hi)
    X = dev(gaussian_states(mu, cb, 16384, lo, hi, seed=24, inflate=2.0))
    f = bm.Forward(model, 4096, binned=True)
    nb = model.n_bins
    Y = torch.empty(X.shape[0], nb, dtype=torch.float64, device="cuda")
    for s0 in range(0, X.shape[0], 4096):
        f(X[s0:s0 + 4096].contiguous())
        Y[s0:s0 + 4096] = f.binned.view(4096, nb)
    mean, scale = standardisation(Y)
    net = MLP([PRIOR.lo.size, 256, 256, 256, nb], max_batch=4096, seed=5)
    tr = Trainer(net, dev(lo), dev(hi), X, Y, mean, scale, batch=256, seed=6)
    for e in range(25):
        tr.epoch(1e-6 + 0.5 * (2e-3 - 1e-6) * (1 + math.cos(math.pi * e / 25)))
    sur = Surrogate(net, dev(lo), dev(hi), mean, scale, model.data, model.err, n_chains=4096)
    x0, z0 = rb.s.x.clone(), rb.s.z[:rb.s.archive_size].clone()

    def production(surrogate):
        r = Retrieval(model, C, PRIOR.lo, PRIOR.hi, seed=31, thin=5, hist_cap=n_gen,
                      surrogate=surrogate, z_cap=z0.shape[0] + C * (n_gen // 5 + 1))
        r.resume(x0, z0)
        r.run(n_gen)
        torch.cuda.synchronize()
        return r.s.n_accept.sum(0).cpu().numpy(), r.s.history.cpu().numpy()

    acc_p, h_p = production(None)
    acc_d, h_d = production(sur)
    exact_plain = C * n_gen                  # every proposal needs the exact model
    exact_da = int(acc_d[0])                 # only stage-1 survivors do
    assert acc_p[1] > 50
    assert exact_da < 0.5 * exact_plain, (exact_da, exact_plain)
    assert acc_d[1] > 0.5 * acc_p[1], (acc_d, acc_p)
    # posterior location agrees between the two runs (short chains: loose bound)
    hp, hd = h_p[n_gen // 2:].reshape(-1, PRIOR.lo.size), h_d[n_gen // 2:].reshape(-1, PRIOR.lo.size)
    assert np.all(np.abs(hd.mean(0) - hp.mean(0)) < 1.0 * hp.std(0) + 1e-12)


def test_monitored_run_checkpoints_and_resumes(tmp_path):
    # Sec. 5's cadence: parts of the run with Gelman-Rubin of the kept samples after each,
    # SPEIS and ESS at the end; a run stopped at a save and resumed from the file
    # reproduces the uninterrupted run exactly (draws are addressed by generation)
    model, _ = _retrieval_setup()
    full = Retrieval(model, 32, PRIOR.lo, PRIOR.hi, seed=321, thin=2, hist_cap=40)
    full.start()
    out = full.run_monitored(40, burn=10, n_saves=4, chunk=5)
    assert [e["generation"] for e in out["log"]] == [10, 20, 30, 40]
    assert "gr_max" not in out["log"][0] and np.isfinite(out["log"][-1]["gr_max"])
    assert out["ess"] > 0 and out["speis_max"] >= 1.0
    part = Retrieval(model, 32, PRIOR.lo, PRIOR.hi, seed=321, thin=2, hist_cap=40)
    part.start()
    ck = str(tmp_path / "state.npz")
    part.run_monitored(20, burn=0, n_saves=2, chunk=5, checkpoint=ck)
    resumed = Retrieval(model, 32, PRIOR.lo, PRIOR.hi, seed=321, thin=2, hist_cap=40)
    resumed.load(ck)
    assert resumed.s.generation == 20
    resumed.run(20)
    torch.cuda.synchronize()
    m = full.s.archive_size
    assert resumed.s.archive_size == m
    assert torch.equal(resumed.s.x, full.s.x) and torch.equal(resumed.s.lp, full.s.lp)
    assert torch.equal(resumed.s.history, full.s.history)
    assert torch.equal(resumed.s.z[:m], full.s.z[:m])
