"""GPU surrogate kernels against the reference MLP: the BF16 matrix-core GEMM in every
epilogue and operand layout, the forward pass and back-propagation layer by layer,
Adam, the surrogate chi^2, and training that reduces the loss."""
import numpy as np
import pytest

from oracle import mlp as om

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import ctypes as C  # noqa: E402

import paper_2104_12522_amd as bm  # noqa: E402
from paper_2104_12522_amd import _abi  # noqa: E402
from paper_2104_12522_amd.surrogate import MLP, Surrogate, Trainer  # noqa: E402

ULP = 2.0 ** -7          # BF16 spacing relative to the leading binade


def to_bf16_dev(x: np.ndarray) -> torch.Tensor:
    """Raw BF16 bit patterns (int16 device tensor) of the oracle's BF16 rounding of x."""
    r = om.bf16(x).astype(np.float32)
    return torch.as_tensor((r.view(np.uint32) >> 16).astype(np.uint16).view(np.int16), device="cuda")


def from_bf16(t: torch.Tensor) -> np.ndarray:
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def gemm(M, N, K, A, lda, ta, B, ldb, tb, mode, bias=None, aux=None, ldaux=0, out=None, ldo=0,
         out16=None, ldob=0, beta=0.0):
    st = bm.lib().bm_gemm_bf16(M, N, K, bm._ptr(A), lda, ta, bm._ptr(B), ldb, tb, mode,
                               bm._ptr(bias), bm._ptr(aux), ldaux, bm._ptr(out), ldo,
                               bm._ptr(out16), ldob, C.c_float(beta), bm._stream())
    bm._check(st, "bm_gemm_bf16")


def _bound(a, b):
    """FP32-accumulation error bound of a @ b."""
    return 2e-6 * np.sqrt(a.shape[1]) * (np.abs(a) @ np.abs(b)) + 1e-30


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("M,N,K", [(70, 130, 45), (1, 1, 1), (128, 64, 96), (33, 1000, 512), (40, 200, 300),
                                   (1024, 1040, 72), (1030, 1030, 45)])
def test_gemm_store_all_layouts(M, N, K, ta, tb):
    g = np.random.default_rng(M * 7 + N + K + 10 * ta + 20 * tb)
    a = om.bf16(g.normal(0, 1, (M, K)))
    b = om.bf16(g.normal(0, 1, (K, N)))
    A = to_bf16_dev(a.T.copy() if ta else a)
    B = to_bf16_dev(b.copy() if tb else b.T.copy())
    out = torch.full((M, N), 7.0, dtype=torch.float32, device="cuda")
    gemm(M, N, K, A, M if ta else K, ta, B, N if tb else K, tb, _abi.BM_GEMM_STORE, out=out, ldo=N)
    ref = a @ b
    assert np.all(np.abs(out.cpu().numpy() - ref) <= _bound(a, b))
    # accumulate: out = 1 * out + a b
    gemm(M, N, K, A, M if ta else K, ta, B, N if tb else K, tb, _abi.BM_GEMM_STORE, out=out, ldo=N,
         beta=1.0)
    assert np.all(np.abs(out.cpu().numpy() - 2 * ref) <= 2 * _bound(a, b))


def test_gemm_bias_silu_and_silu_grad_epilogues():
    M, N, K = 100, 200, 80
    g = np.random.default_rng(3)
    a, w = om.bf16(g.normal(0, 1, (M, K))), om.bf16(g.normal(0, 0.2, (N, K)))
    bias = g.normal(0, 0.5, N).astype(np.float32)
    A, W = to_bf16_dev(a), to_bf16_dev(w)
    z = torch.empty(M, N, dtype=torch.float32, device="cuda")
    h = torch.empty(M, N, dtype=torch.int16, device="cuda")
    bt = torch.as_tensor(bias, device="cuda")
    gemm(M, N, K, A, K, 0, W, K, 0, _abi.BM_GEMM_BIAS_SILU, bias=bt, out=z, ldo=N, out16=h, ldob=N)
    zr = a @ w.T + bias
    zg = z.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(zg - zr) <= _bound(a, w.T) + 1e-6 * np.abs(bias))
    np.testing.assert_allclose(from_bf16(h), om.bf16(om.silu(zg)), rtol=ULP, atol=1e-30)
    # linear epilogue
    lin = torch.empty(M, N, dtype=torch.float32, device="cuda")
    gemm(M, N, K, A, K, 0, W, K, 0, _abi.BM_GEMM_BIAS, bias=bt, out=lin, ldo=N)
    np.testing.assert_array_equal(lin.cpu().numpy(), z.cpu().numpy())
    # dX * silu'(aux) with aux the pre-activations above
    d = om.bf16(g.normal(0, 1, (M, N)))
    D = to_bf16_dev(d)
    dx = torch.empty(M, K, dtype=torch.int16, device="cuda")
    gemm(M, K, N, D, N, 0, W, K, 1, _abi.BM_GEMM_SILU_GRAD, aux=z[:, :K].contiguous(), ldaux=K,
         out16=dx, ldob=K)
    raw = d @ w
    ref = raw * om.silu_grad(zg[:, :K])
    got = from_bf16(dx)
    tol = ULP * np.abs(ref) + _bound(d, w) * np.abs(om.silu_grad(zg[:, :K])) * 2
    assert np.all(np.abs(got - ref) <= tol)


def test_gemm_rejects_bad_arguments():
    A = torch.zeros(4, dtype=torch.int16, device="cuda")
    out = torch.zeros(4, dtype=torch.float32, device="cuda")
    lib = bm.lib()
    s = bm._stream()
    assert lib.bm_gemm_bf16(2, 2, 2, bm._ptr(A), 2, 0, bm._ptr(A), 2, 0, 9, None, None, 0,
                            bm._ptr(out), 2, None, 0, C.c_float(0), s) == _abi.BM_EINVAL
    assert lib.bm_gemm_bf16(2, 2, 2, bm._ptr(A), 2, 0, bm._ptr(A), 2, 0, _abi.BM_GEMM_BIAS_SILU,
                            None, None, 0, bm._ptr(out), 2, None, 0, C.c_float(0), s) == _abi.BM_EINVAL
    assert lib.bm_gemm_bf16(-1, 2, 2, bm._ptr(A), 2, 0, bm._ptr(A), 2, 0, 0, None, None, 0,
                            bm._ptr(out), 2, None, 0, C.c_float(0), s) == _abi.BM_ESHAPE


DIMS = [10, 64, 96, 64, 40]
LO = np.array([-3, -1.5, -1.5, 0, 0.6, -8, -8, -8, -8, 1.0])
HI = np.array([0, 1, 1, 1, 1.2, -2, -2, -2, -2, 1.3])


def _net_and_input(B=37, seed=0):
    net = MLP(DIMS, max_batch=64, seed=seed)
    g = np.random.default_rng(seed + 1)
    for b in net.b32:
        b.copy_(torch.as_tensor(g.normal(0, 0.1, b.numel()).astype(np.float32)))
    params = torch.as_tensor(LO + (HI - LO) * g.random((B, 10)), device="cuda")
    lo, hi = torch.as_tensor(LO, device="cuda"), torch.as_tensor(HI, device="cuda")
    return net, params, lo, hi


def test_input_scaling_and_row_gather():
    net, params, lo, hi = _net_and_input()
    rows = torch.tensor([5, 0, 36, 5], dtype=torch.int32, device="cuda")
    net.set_input(params, lo, hi, rows=rows, B=4)
    torch.cuda.synchronize()
    ref = om.bf16(om.scale_input(params.cpu().numpy()[[5, 0, 36, 5]], LO, HI))
    np.testing.assert_array_equal(from_bf16(net.h[0][:4]), ref)


def test_forward_layer_by_layer_matches_oracle():
    B = 37
    net, params, lo, hi = _net_and_input(B)
    out = torch.empty(B, DIMS[-1], dtype=torch.float32, device="cuda")
    net.set_input(params, lo, hi)
    net.forward(B, out)
    torch.cuda.synchronize()
    for i in range(net.n_layers):
        h = from_bf16(net.h[i][:B])
        w = from_bf16(net.w16[i])
        np.testing.assert_array_equal(w, om.bf16(net.w32[i].cpu().numpy()))
        zr = h @ w.T + net.b32[i].cpu().numpy()
        zg = (net.z[i][:B] if i < net.n_layers - 1 else out).cpu().numpy().astype(np.float64)
        assert np.all(np.abs(zg - zr) <= _bound(h, w.T) + 1e-6 * np.abs(zr))
        if i < net.n_layers - 1:
            np.testing.assert_allclose(from_bf16(net.h[i + 1][:B]), om.bf16(om.silu(zg)), rtol=ULP)
    # end to end against the FP64 network with the same BF16 weights
    ws = [om.bf16(w.cpu().numpy()) for w in net.w32]
    bs = [b.cpu().numpy().astype(np.float64) for b in net.b32]
    _, _, ref = om.forward(om.scale_input(params.cpu().numpy(), LO, HI), ws, bs)
    g = out.cpu().numpy()
    assert np.sqrt(np.mean((g - ref) ** 2)) < 2e-2 * np.sqrt(np.mean(ref ** 2))


def test_backward_matches_oracle_gradients():
    B = 48
    net, params, lo, hi = _net_and_input(B, seed=5)
    g = np.random.default_rng(9)
    target = torch.as_tensor(g.normal(0, 1, (B, DIMS[-1])), device="cuda")
    out = torch.empty(B, DIMS[-1], dtype=torch.float32, device="cuda")
    row_loss = torch.empty(B, dtype=torch.float32, device="cuda")
    net.set_input(params, lo, hi)
    net.forward(B, out)
    net.loss_grad(B, out, target, row_loss=row_loss)
    torch.cuda.synchronize()
    o = out.cpu().numpy().astype(np.float64)
    t = target.cpu().numpy()
    np.testing.assert_allclose(row_loss.cpu().numpy(), ((o - t) ** 2).sum(1), rtol=1e-5)
    dout = from_bf16(net.dz[0].view(-1)[:B * DIMS[-1]].view(B, DIMS[-1]))   # dz rows have stride N
    np.testing.assert_allclose(dout, om.bf16(om.mse_grad(o, t)), rtol=ULP, atol=1e-30)
    net.backward(B)
    torch.cuda.synchronize()
    hs = [from_bf16(h[:B]) for h in net.h]
    zs = [z[:B].cpu().numpy().astype(np.float64) for z in net.z[:-1]] + [o]
    ws = [from_bf16(w) for w in net.w16]
    gw_r, gb_r = om.backward(ws, zs, hs, dout, round_bf16=True)
    # same-precision reference: a BF16 flip of one back-propagated element moves one term
    # of a batch sum by at most one BF16 spacing
    dz = dout
    for i in range(net.n_layers - 1, -1, -1):
        gw = net.gw[i].cpu().numpy()
        gb = net.gb[i].cpu().numpy()
        scale_w = np.abs(dz).T @ np.abs(hs[i])
        assert np.all(np.abs(gw - gw_r[i]) <= 2 * ULP * scale_w + 1e-30), i
        assert np.all(np.abs(gb - gb_r[i]) <= 2 * ULP * np.abs(dz).sum(0) + 1e-30), i
        if i > 0:
            dz = om.bf16((dz @ ws[i]) * om.silu_grad(zs[i - 1]))
    # and against exact FP64 back-propagation of the FP64 network
    w64 = [w.cpu().numpy().astype(np.float64) for w in net.w32]
    b64 = [b.cpu().numpy().astype(np.float64) for b in net.b32]
    zs64, hs64, o64 = om.forward(om.scale_input(params.cpu().numpy(), LO, HI), w64, b64)
    gw64, _ = om.backward(w64, zs64, hs64, om.mse_grad(o64, t))
    for i in range(net.n_layers):
        a, b = net.gw[i].cpu().numpy().ravel(), gw64[i].ravel()
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        assert cos > 0.995, (i, cos)


def test_adam_step_matches_oracle():
    net, _, _, _ = _net_and_input()
    g = np.random.default_rng(11)
    w0 = [w.cpu().numpy().astype(np.float64) for w in net.w32]
    b0 = [b.cpu().numpy().astype(np.float64) for b in net.b32]
    m = [np.zeros_like(w) for w in w0]
    v = [np.zeros_like(w) for w in w0]
    mb = [np.zeros_like(b) for b in b0]
    vb = [np.zeros_like(b) for b in b0]
    for step in range(1, 4):
        grads = [g.normal(0, 1e-2, w.shape).astype(np.float32) for w in w0]
        gbs = [g.normal(0, 1e-2, b.shape).astype(np.float32) for b in b0]
        for i in range(net.n_layers):
            net.gw[i].copy_(torch.as_tensor(grads[i]))
            net.gb[i].copy_(torch.as_tensor(gbs[i]))
        net.adam(1e-3)
        torch.cuda.synchronize()
        for i in range(net.n_layers):
            w0[i], m[i], v[i] = om.adam(w0[i], grads[i].astype(np.float64), m[i], v[i], step, 1e-3)
            b0[i], mb[i], vb[i] = om.adam(b0[i], gbs[i].astype(np.float64), mb[i], vb[i], step, 1e-3)
            # FP32 storage of w each step plus a relative 1e-6 on the update (lr = 1e-3)
            tol_w = step * 2.0 ** -23 * np.abs(w0[i]) + step * 1e-9
            tol_b = step * 2.0 ** -23 * np.abs(b0[i]) + step * 1e-9
            assert np.all(np.abs(net.w32[i].cpu().numpy() - w0[i]) <= tol_w)
            assert np.all(np.abs(net.b32[i].cpu().numpy() - b0[i]) <= tol_b)
            np.testing.assert_array_equal(from_bf16(net.w16[i]), om.bf16(net.w32[i].cpu().numpy()))


def test_surrogate_chi2_matches_oracle():
    net, params, lo, hi = _net_and_input(20)
    g = np.random.default_rng(12)
    N = DIMS[-1]
    mean, scale = g.normal(0.015, 1e-3, N), g.uniform(1e-4, 1e-3, N)
    data, err = g.normal(0.015, 1e-3, N), np.full(N, 6e-5)
    dev = lambda a: torch.as_tensor(a, device="cuda")  # noqa: E731
    s = Surrogate(net, lo, hi, dev(mean), dev(scale), dev(data), dev(err), n_chains=20)
    chi2 = s(params).cpu().numpy()
    out = s.out[:20].cpu().numpy()
    np.testing.assert_allclose(chi2, om.surrogate_chi2(out, mean, scale, data, err), rtol=1e-12)


def test_training_reduces_loss_on_smooth_targets():
    g = np.random.default_rng(13)
    n, N = 4096, 40
    theta = LO + (HI - LO) * g.random((n, 10))
    x = om.scale_input(theta, LO, HI)
    proj = g.normal(0, 1, (10, N))
    y = np.sin(x @ proj) + 0.5 * (x @ proj) ** 2 / 10
    mean, scale = y.mean(0), y.std(0)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")  # noqa: E731
    net = MLP([10, 128, 128, N], max_batch=256, seed=1)
    tr = Trainer(net, dev(LO), dev(HI), dev(theta), dev(y), dev(mean), dev(scale), batch=256, seed=2)
    first = float(tr.epoch(3e-3).mean()) / N
    for e in range(60):
        last = float(tr.epoch(3e-3 if e < 40 else 1e-3).mean()) / N
    assert np.isfinite(last) and last < first / 20, (first, last)
