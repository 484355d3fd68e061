"""Placement MLP: the oracle pinned by finite differences; the library's host
forward pass, BF16 rounding and learned planner on the CPU; and (GPU) the
hand-written training and inference kernels against the oracle."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import mlp as om

lms = pytest.importorskip("paper_2111_04289_amd.lms")


def rand_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, om.NPARAMS)


def rand_data(seed, n):
    rng = np.random.default_rng(seed)
    x = rng.normal(0, 1, (n, 12))
    t = rng.normal(0, 1, (n, 2))
    m = (rng.random((n, 2)) < 0.8).astype(np.float64)
    return x, t, m


def test_oracle_gradient_matches_central_differences():
    p = rand_params(0)
    x, t, m = rand_data(1, 9)
    _, g = om.loss_grad(p, x, t, m)
    rng = np.random.default_rng(2)
    idx = rng.choice(om.NPARAMS, 300, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (om.loss(p + e, x, t, m) - om.loss(p - e, x, t, m)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i


def test_oracle_loss_masks_and_averages():
    p = rand_params(3)
    x, t, m = rand_data(4, 5)
    y, _ = om.forward(p, x)
    m0 = np.zeros_like(m)
    assert om.loss(p, x, t, m0) == 0.0
    m1 = np.zeros_like(m)
    m1[2, 1] = 1
    assert om.loss(p, x, t, m1) == pytest.approx((y[2, 1] - t[2, 1]) ** 2 / 5)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(5)
    xs = np.concatenate([rng.normal(0, 10, 2000), [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -0.0, 65504.0, 1e-38]])
    xs = xs.astype(np.float32)
    ref = torch.from_numpy(xs).to(torch.bfloat16).float().numpy()
    got = np.array([lms._lib.lms_bf16_round(ctypes.c_float(float(v))) for v in xs], np.float32)
    np.testing.assert_array_equal(got, ref)


def test_host_forward_matches_oracle():
    p = rand_params(6)
    x, _, _ = rand_data(7, 20)
    y, _ = om.forward(p, x)
    pf = p.astype(np.float32)
    for s in range(20):
        out = np.zeros(2, np.float32)
        lms._lib.lms_mlp_host_forward(pf.ctypes.data_as(ctypes.c_void_p), x[s].astype(np.float32).ctypes.data_as(
            ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p))
        np.testing.assert_allclose(out, y[s], rtol=2e-4, atol=2e-4)


def test_features_layout():
    f = lms.mlp_features(lms.OP_AGG, rows=(1 << 20) - 1, ncols=4, selectivity=0.3, distinct_keys=1023,
                         window_s=10, slide_s=1, interval_s=2.5, transfer=1)
    assert f[0] == pytest.approx(20 / 24)
    assert f[1] == pytest.approx(0.5) and f[2] == pytest.approx(0.3) and f[3] == pytest.approx(10 / 20)
    assert list(f[4:8]) == [0, 0, 1, 0]  # sliding aggregation
    assert f[8] == pytest.approx(10 / 60) and f[9] == pytest.approx(1 / 60) and f[10] == pytest.approx(0.25)
    assert f[11] == 1
    g = lms.mlp_features(lms.OP_AGG, rows=1, ncols=1, selectivity=1, distinct_keys=0, window_s=5, slide_s=0,
                         interval_s=0, transfer=0)
    assert list(g[4:8]) == [0, 1, 0, 0]  # tumbling aggregation
    assert list(lms.mlp_features(lms.OP_JOIN, 1, 1, 1, 0, 0, 0, 0, 0)[4:8]) == [0, 0, 0, 1]
    assert list(lms.mlp_features(lms.OP_FILTER, 1, 1, 1, 0, 0, 0, 0, 0)[4:8]) == [1, 0, 0, 0]


def test_learned_plan_picks_smaller_prediction():
    # a model whose output ignores x except through the transfer flag (x11):
    # log GPU ms = 0.5 + 2 * x11, log CPU ms = 1.0
    d = {name: np.zeros(shape) for name, shape in om.SIZES}
    d["W1"][0, 11] = 1.0  # h1[0] = transfer flag
    d["W2"][0, 0] = 1.0   # h2[0] = h1[0]
    d["W3"][1, 0] = 2.0
    d["b3"][:] = [1.0, 0.5]
    p = om.pack(d).astype(np.float32)
    kinds = [lms.OP_SCAN, lms.OP_FILTER, lms.OP_PROJECT, lms.OP_AGG]
    devs, costs = lms.lms_plan(kinds, 10 * 153600, 1, mode=lms.PLAN_LEARNED, model=p)
    # first op: transfer -> GPU 2.5 > CPU 1.0 -> CPU; next: prev on CPU -> transfer -> CPU; ... last -> CPU
    assert devs == [lms.DEV_CPU] * 4
    assert costs == pytest.approx([np.e] * 4, rel=1e-6)
    d["b3"][:] = [3.0, 0.5]  # CPU now slower than GPU even with transfer
    devs, costs = lms.lms_plan(kinds, 10 * 153600, 1, mode=lms.PLAN_LEARNED, model=om.pack(d).astype(np.float32))
    assert devs == [lms.DEV_GPU] * 4
    # first and last ops pay the transfer (exp 2.5), the middle ones do not (exp 0.5)
    assert costs == pytest.approx([np.exp(2.5), np.exp(0.5), np.exp(0.5), np.exp(2.5)], rel=1e-6)


# ------------------------------------------------------------------ GPU kernels

@pytest.mark.gpu
@pytest.mark.parametrize("n", [1, 63, 64, 1000, 4097])
def test_gpu_loss_grad_matches_oracle(n):
    p = rand_params(10 + n)
    x, t, m = rand_data(20 + n, n)
    net = lms.Mlp(seed=1)
    net.set_params(p.astype(np.float32))
    L, g = net.loss_grad(*(torch.from_numpy(a.astype(np.float32)).cuda() for a in (x, t, m)))
    # the oracle runs on the FP32-rounded parameters and inputs the kernel sees
    Lo, go = om.loss_grad(p.astype(np.float32), x.astype(np.float32), t.astype(np.float32), m.astype(np.float32))
    assert L == pytest.approx(Lo, rel=1e-4)
    np.testing.assert_allclose(g, go, rtol=1e-3, atol=1e-5 * max(1.0, np.abs(go).max()))


@pytest.mark.gpu
def test_gpu_forward_fp32_and_bf16():
    p = rand_params(30).astype(np.float32)
    x, _, _ = rand_data(31, 3000)
    net = lms.Mlp(seed=1)
    net.set_params(p)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    y32 = net.forward(xd).cpu().numpy()
    yo, _ = om.forward(p, x.astype(np.float32))
    np.testing.assert_allclose(y32, yo, rtol=2e-4, atol=2e-4)
    yb = net.forward(xd, bf16=True).cpu().numpy()
    pb = torch.from_numpy(p).to(torch.bfloat16).float().numpy()
    yob, _ = om.forward(pb, x.astype(np.float32))
    np.testing.assert_allclose(yb, yob, rtol=2e-4, atol=2e-4)


@pytest.mark.gpu
def test_gpu_adam_matches_oracle_and_training_fits():
    p = rand_params(40, 0.2).astype(np.float32)
    x, t, m = rand_data(41, 2000)
    t = np.stack([np.sin(x[:, 0]) + 0.5 * x[:, 1], x[:, 2] * x[:, 3]], 1)  # a learnable target
    net = lms.Mlp(seed=1)
    net.set_params(p)
    X, T, M = (torch.from_numpy(a.astype(np.float32)).cuda() for a in (x, t, m))
    po, mo, vo = p.astype(np.float64), np.zeros(om.NPARAMS), np.zeros(om.NPARAMS)
    for step in range(1, 4):
        L, g = net.loss_grad(X, T, M)
        net.adam(lr=1e-3)
        _, go = om.loss_grad(po.astype(np.float32), x.astype(np.float32), t.astype(np.float32), m.astype(np.float32))
        po, mo, vo = om.adam(po, go, mo, vo, step, 1e-3)
        np.testing.assert_allclose(net.get_params(), po, rtol=1e-3, atol=1e-4)
    first = None
    for step in range(300):
        L, _ = net.loss_grad(X, T, M)
        net.adam(lr=3e-3)
        first = L if first is None else first
    assert L < 0.3 * first
