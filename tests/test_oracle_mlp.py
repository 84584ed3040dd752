"""Pins of the reference MLP surrogate: BF16 rounding against an independent converter
and hand-checked ties, SiLU and back-propagation against central finite differences,
Adam against its closed form under a constant gradient."""
import numpy as np
import pytest

from oracle import mlp as om


def test_bf16_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(0)
    x = np.concatenate([g.normal(0, 1, 5000), g.normal(0, 1e-30, 500), g.normal(0, 1e30, 500),
                        [0.0, -0.0, np.inf, -np.inf, 1e-40, 3.4e38]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(om.bf16(x), ref)


def test_bf16_ties_round_to_even():
    # 7 fraction bits: the spacing above 1 is 2^-7
    assert om.bf16(1 + 2.0 ** -8)[()] == 1.0                      # tie, 1.0 is even
    assert om.bf16(1 + 3 * 2.0 ** -8)[()] == 1 + 2.0 ** -6         # tie, up to the even one
    assert om.bf16(1 + 2.0 ** -8 + 2.0 ** -20)[()] == 1 + 2.0 ** -7  # above the tie
    assert np.isnan(om.bf16(np.nan))


def test_silu_values_and_derivative():
    assert om.silu(0.0) == 0.0
    assert om.silu(40.0) == pytest.approx(40.0)
    assert om.silu(-40.0) == pytest.approx(0.0, abs=1e-15)
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    fd = (om.silu(z + h) - om.silu(z - h)) / (2 * h)
    np.testing.assert_allclose(om.silu_grad(z), fd, rtol=1e-8, atol=1e-10)
    assert om.silu_grad(0.0) == pytest.approx(0.5)


def _net(dims, seed):
    g = np.random.default_rng(seed)
    ws = [g.normal(0, 1 / np.sqrt(dims[i]), (dims[i + 1], dims[i])) for i in range(len(dims) - 1)]
    bs = [g.normal(0, 0.1, dims[i + 1]) for i in range(len(dims) - 1)]
    return ws, bs


@pytest.mark.parametrize("dims", [[3, 2], [4, 6, 5, 3], [10, 8, 8, 8, 8, 7]])
def test_backward_matches_finite_differences(dims):
    g = np.random.default_rng(1)
    ws, bs = _net(dims, 2)
    x = g.uniform(0, 1, (5, dims[0]))
    t = g.normal(0, 1, (5, dims[-1]))

    def loss(ws_, bs_):
        return om.mse(om.forward(x, ws_, bs_)[2], t)
    zs, hs, out = om.forward(x, ws, bs)
    gw, gb = om.backward(ws, zs, hs, om.mse_grad(out, t))
    h = 1e-6
    for i in range(len(ws)):
        for idx in [(0, 0), (ws[i].shape[0] - 1, ws[i].shape[1] - 1), (ws[i].shape[0] // 2, 0)]:
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[i][idx] += h
            wm[i][idx] -= h
            fd = (loss(wp, bs) - loss(wm, bs)) / (2 * h)
            assert gw[i][idx] == pytest.approx(fd, rel=1e-6, abs=1e-10)
        for j in [0, bs[i].size - 1]:
            bp = [b.copy() for b in bs]
            bm_ = [b.copy() for b in bs]
            bp[i][j] += h
            bm_[i][j] -= h
            fd = (loss(ws, bp) - loss(ws, bm_)) / (2 * h)
            assert gb[i][j] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_linear_layer_gradient_is_least_squares_normal_equation():
    # one linear layer: the gradient vanishes exactly at the least-squares solution
    g = np.random.default_rng(3)
    x = g.normal(0, 1, (40, 3))
    t = g.normal(0, 1, (40, 2))
    xa = np.hstack([x, np.ones((40, 1))])
    sol = np.linalg.lstsq(xa, t, rcond=None)[0]
    w, b = sol[:3].T.copy(), sol[3].copy()
    zs, hs, out = om.forward(x, [w], [b])
    gw, gb = om.backward([w], zs, hs, om.mse_grad(out, t))
    assert np.abs(gw[0]).max() < 1e-13 and np.abs(gb[0]).max() < 1e-13


def test_adam_constant_gradient_closed_form():
    # with a constant gradient the bias-corrected moments are g and g^2 at every step,
    # so each step moves w by lr * g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    w, m, v = np.array([1.0, 2.0, 3.0, 4.0]), np.zeros(4), np.zeros(4)
    lr, eps = 0.01, 1e-8
    w0 = w.copy()
    for step in range(1, 6):
        w, m, v = om.adam(w, g, m, v, step, lr, eps=eps)
        np.testing.assert_allclose(w, w0 - step * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_surrogate_chi2_of_exact_standardised_spectrum():
    g = np.random.default_rng(4)
    mean, scale = g.normal(0.015, 1e-3, 50), g.uniform(1e-4, 1e-3, 50)
    spec = g.normal(0.015, 1e-3, 50)
    data = spec + g.normal(0, 6e-5, 50)
    err = np.full(50, 6e-5)
    out = (spec - mean) / scale
    assert om.surrogate_chi2(out, mean, scale, data, err)[0] == pytest.approx(
        np.sum(((spec - data) / err) ** 2), rel=1e-10)


def test_bf16_forward_is_exact_for_representable_operands():
    # operands already in BF16: rounding changes nothing, so the two passes agree
    g = np.random.default_rng(5)
    ws = [om.bf16(g.normal(0, 0.5, (4, 3))), om.bf16(g.normal(0, 0.5, (2, 4)))]
    bs = [np.zeros(4), np.zeros(2)]
    x = om.bf16(g.uniform(0, 1, (6, 3)))
    zs_r, _, _ = om.forward(x, ws, bs, round_bf16=True)
    zs, _, _ = om.forward(x, ws, bs)
    np.testing.assert_array_equal(zs_r[0], zs[0])
