"""Pins for the FP64 reference network: layers against torch's CPU convolutions, gradients
against central finite differences, BF16 rounding against torch's bfloat16 conversion."""
import numpy as np
import pytest
import torch

import inputs
from oracle import nn_ref


def _params(seed=1, scale=1.0):
    p = []
    for name, shp in nn_ref.SHAPES:
        n = int(np.prod(shp))
        fan = shp[1] * shp[2] * shp[3] if name in ("W0", "W1") else (shp[0] * shp[2] * shp[3] if len(shp) == 4 else 1)
        bound = scale * np.sqrt(6.0 / fan)
        p.append(inputs.uniform(seed, len(p), n, -bound, bound) if len(shp) == 4 else
                 inputs.uniform(seed, len(p), n, -0.05, 0.05))
    return np.concatenate(p)


def test_layers_match_torch_cpu():
    p = _params()
    P = nn_ref.unpack(p)
    x = inputs.normal(3, 0, 2 * 2 * 32 * 32).reshape(2, 2, 32, 32)
    y, c = nn_ref.forward(p, x, bf=False)
    xt = torch.tensor(x)
    z1 = torch.nn.functional.conv2d(xt, torch.tensor(P["W0"]), torch.tensor(P["b0"]), padding=1).relu()
    z2 = torch.nn.functional.conv2d(z1, torch.tensor(P["W1"]), torch.tensor(P["b1"]), stride=2, padding=1).relu()
    z2 = z2 + z2.mean(dim=(2, 3), keepdim=True)
    z3 = torch.nn.functional.conv_transpose2d(z2, torch.tensor(P["W2"]), torch.tensor(P["b2"]), stride=4).relu()
    yt = torch.nn.functional.conv_transpose2d(z3, torch.tensor(P["W3"]), torch.tensor(P["b3"]), stride=1)
    assert yt.shape == (2, 1, 65, 65)
    assert np.allclose(y, yt.reshape(2, -1).numpy(), rtol=1e-12, atol=1e-12)


def test_bf16_rounding_matches_torch():
    v = inputs.normal(4, 0, 10000) * 10.0 ** inputs.uniform(4, 1, 10000, -3, 3)
    ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(nn_ref.bf16(v), ref)


@pytest.mark.parametrize("w", [0.0, 0.3])
def test_gradient_matches_central_differences(w):
    p = _params(2, scale=0.7)
    x = inputs.normal(5, 0, 2 * 32 * 32).reshape(1, 2, 32, 32)
    t = inputs.normal(6, 0, 65 * 65).reshape(1, -1)
    _, g = nn_ref.loss_and_grad(p, x, t, bf=False, lap_weight=w)
    idx = np.concatenate([np.arange(0, nn_ref.NPARAM, 4999), [nn_ref.NPARAM - 1, nn_ref.NPARAM - 2]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = nn_ref.loss_and_grad(p + e, x, t, bf=False, lap_weight=w)
        lm, _ = nn_ref.loss_and_grad(p - e, x, t, bf=False, lap_weight=w)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])
