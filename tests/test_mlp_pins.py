"""Pins of the placement-MLP oracle (oracle/mlp.py) against an independent
implementation: torch's CPU layers, autograd and optimizer in float64.

The parameter layout is taken from its definition in the C header (W1[64][12],
b1[64], W2[64][64], b2[64], W3[2][64], b3[2], row-major, W[out][in]), not from
the oracle's own unpacking, so a layout slip made consistently in the oracle's
forward pass and its gradient (which finite differences cannot see) fails
here.  Planted mistakes (a transposed W2 in both passes, Adam without bias
correction) must each be rejected by these pins.
"""
import math
import os
import types

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import mlp as om

IN, HID, OUT = 12, 64, 2
LAYOUT = [(HID, IN), (HID,), (HID, HID), (HID,), (OUT, HID), (OUT,)]


def torch_params(p):
    """The flat parameter vector split per the header's layout into leaf tensors."""
    out, o = [], 0
    for shape in LAYOUT:
        k = int(np.prod(shape))
        out.append(torch.tensor(np.asarray(p[o:o + k]), dtype=torch.float64).reshape(shape).requires_grad_(True))
        o += k
    assert o == len(p)
    return out


def torch_forward(ts, x):
    W1, b1, W2, b2, W3, b3 = ts
    h1 = F.relu(F.linear(x, W1, b1))  # y[o] = sum_i W[o][i] x[i] + b[o]
    h2 = F.relu(F.linear(h1, W2, b2))
    return F.linear(h2, W3, b3)


def rand_case(seed, n=17):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, om.NPARAMS)
    x = rng.normal(0, 1, (n, IN))
    t = rng.normal(0, 1, (n, OUT))
    m = (rng.random((n, OUT)) < 0.7).astype(np.float64)
    return p, x, t, m


def check_forward(mod, seed):
    p, x, _, _ = rand_case(seed)
    W2 = p[HID * IN + HID:HID * IN + HID + HID * HID].reshape(HID, HID)
    assert not np.allclose(W2, W2.T)  # a transposed W2 would change the result
    y, _ = mod.forward(p, x)
    with torch.no_grad():
        ref = torch_forward(torch_params(p), torch.tensor(x)).numpy()
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)


def check_loss_grad(mod, seed):
    p, x, t, m = rand_case(seed)
    L, g = mod.loss_grad(p, x, t, m)
    ts = torch_params(p)
    y = torch_forward(ts, torch.tensor(x))
    loss = (torch.tensor(m) * (y - torch.tensor(t)) ** 2).sum() / len(x)
    loss.backward()
    ref = np.concatenate([a.grad.numpy().ravel() for a in ts])
    assert L == pytest.approx(float(loss.detach()), rel=1e-12)
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-12)


def check_adam(mod, seed, steps=3, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 1, 50)
    grads = [rng.normal(0, 1, 50) * 10.0 ** rng.integers(-3, 2, 50) for _ in range(steps)]
    tp = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=lr, betas=(b1, b2), eps=eps)
    q, mm, vv = p.copy(), np.zeros_like(p), np.zeros_like(p)
    for s, g in enumerate(grads, start=1):
        q, mm, vv = mod.adam(q, g, mm, vv, s, lr, b1, b2, eps)
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
        np.testing.assert_allclose(q, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


def check_adam_first_step(mod):
    """Closed form of the first step: m = (1-b1) g and v = (1-b2) g^2 bias-correct
    to g and g^2, so the update is lr * g / (|g| + eps), i.e. lr * sign(g) when
    |g| >> eps, whatever b1 and b2 are."""
    g = np.array([3.0, -0.25, 1e3, -7e-3, 0.5])
    p = np.zeros_like(g)
    for b1, b2 in ((0.9, 0.999), (0.5, 0.9)):
        q, _, _ = mod.adam(p, g, np.zeros_like(g), np.zeros_like(g), 1, 0.01, b1, b2, 1e-8)
        np.testing.assert_allclose(q, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
        np.testing.assert_allclose(np.abs(q), 0.01, rtol=2e-6)


@pytest.mark.parametrize("seed", range(3))
def test_forward_matches_torch_linear_layers(seed):
    check_forward(om, seed)


@pytest.mark.parametrize("seed", range(3))
def test_loss_grad_matches_torch_autograd(seed):
    check_loss_grad(om, seed)


@pytest.mark.parametrize("seed", range(3))
def test_adam_matches_torch_optim(seed):
    check_adam(om, seed)


def test_adam_first_step_closed_form():
    check_adam_first_step(om)


# ---- planted mistakes -------------------------------------------------------------

MUTANTS = {
    # W2 used transposed, consistently in the forward pass and in backpropagation
    # (its finite-difference gradient check still passes)
    "w2_transposed": [('z2 = h1 @ w["W2"].T + w["b2"]', 'z2 = h1 @ w["W2"] + w["b2"]'),
                      ('g["W2"] = dz2.T @ h1', 'g["W2"] = (dz2.T @ h1).T'),
                      ('dz1 = (dz2 @ w["W2"])', 'dz1 = (dz2 @ w["W2"].T)')],
    "adam_no_bias_correction": [("mh = m / (1 - b1 ** step)", "mh = m"), ("vh = v / (1 - b2 ** step)", "vh = v")],
    "adam_no_first_moment_correction": [("mh = m / (1 - b1 ** step)", "mh = m")],
    "relu_on_output": [('y = h2 @ w["W3"].T + w["b3"]', 'y = np.maximum(h2 @ w["W3"].T + w["b3"], 0.0)')],
}


def mutant(name):
    text = open(os.path.join(os.path.dirname(om.__file__), "mlp.py")).read()
    for old, new in MUTANTS[name]:
        assert text.count(old) == 1, f"mutation anchor {old!r} vanished from the oracle source"
        text = text.replace(old, new)
    mod = types.ModuleType(f"mlp_{name}")
    exec(compile(text, f"mlp_{name}.py", "exec"), mod.__dict__)
    return mod


def battery(mod):
    failures = []
    checks = [lambda: check_forward(mod, 0), lambda: check_loss_grad(mod, 1), lambda: check_adam(mod, 2),
              lambda: check_adam_first_step(mod)]
    for c in checks:
        try:
            c()
        except AssertionError as e:
            failures.append(repr(e)[:80])
    return failures


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_planted_mistake(name):
    assert battery(mutant(name)), f"no pin caught the planted mistake {name}"


def test_unmutated_oracle_passes_battery():
    assert battery(om) == []
    assert math.isfinite(om.loss(*rand_case(0)))
