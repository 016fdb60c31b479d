"""Pins of the refiner oracle: bfloat16 rounding on boundary bit patterns and
against torch's conversion, the unrounded MLP against torch autograd, the
identity property of a zero last layer, and the exact inverse relation between
refined_fan and fit_targets."""
import numpy as np
import pytest

from oracle import convert as oc
from oracle import mlp as om
from paper_2502_07754_amd import scenes


def _b(bits):
    return np.array([bits], dtype=np.uint32).view(np.float32)[0]


def test_bf16_rounding_boundaries():
    cases = [
        (1.0, 1.0),
        (1 + 2 ** -8, 1.0),                      # tie -> even (down)
        (1 + 3 * 2 ** -8, 1 + 2 ** -6),          # tie -> even (up)
        (1 + 2 ** -8 + 2 ** -20, 1 + 2 ** -7),   # above the tie
        (-(1 + 3 * 2 ** -8), -(1 + 2 ** -6)),
        (float("inf"), float("inf")),
        (-0.0, -0.0),
        (_b(0x00000001), 0.0),                   # smallest subnormal rounds to zero
        (_b(0x00008000), 0.0),                   # exact tie at the bottom -> even (zero)
        (_b(0x00018000), _b(0x00020000)),        # tie with odd lsb -> up
        (_b(0x7F7FFFFF), float("inf")),          # largest float rounds up to inf
    ]
    for x, want in cases:
        got = om.bf16_round(np.float32(x))
        assert got == want and np.signbit(got) == np.signbit(want), (x, got, want)
    assert np.isnan(om.bf16_round(np.float32("nan")))


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 10000), rng.normal(0, 1e-30, 1000), rng.normal(0, 1e30, 1000)])
    x = x.astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(om.bf16_round(x), want)


def test_mlp_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    p = om.init_params(28, seed=1, zero_last=False)
    rng = np.random.default_rng(2)
    x = rng.normal(size=(40, om.N_IN))
    dy = rng.normal(size=(40, 28))
    y, cache = om.forward(p, x, rounding=False)
    g = om.backward(p, cache, dy, rounding=False)
    t = {k: torch.tensor(v.astype(np.float64), requires_grad=True) for k, v in p.items()}
    xt = torch.tensor(x)
    h1 = torch.relu(xt @ t["W1"].T + t["b1"])
    h2 = torch.relu(h1 @ t["W2"].T + t["b2"])
    yt = h2 @ t["W3"].T + t["b3"]
    (yt * torch.tensor(dy)).sum().backward()
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    for k in p:
        np.testing.assert_allclose(g[k], t[k].grad.numpy(), rtol=1e-10, atol=1e-12)


def test_rounded_forward_is_near_unrounded():
    p = om.init_params(28, seed=3, zero_last=False)
    x = np.random.default_rng(4).normal(size=(64, om.N_IN))
    y0, _ = om.forward(p, x, rounding=False)
    y1, _ = om.forward(p, x, rounding=True)
    rel = np.abs(y1 - y0).max() / np.abs(y0).max()
    assert 1e-4 < rel < 3e-2        # bfloat16 operands: ~2^-8 relative per product


def test_zero_last_layer_is_plain_conversion():
    g = scenes.gaussians(50, 7, 0.01, 0.1, flat=True)
    p = om.init_params(3 * 8 + 4, seed=0, zero_last=True)
    x = om.features(g.mean, g.scale, g.quat, g.opacity, g.rgb, 8)
    y, _ = om.forward(p, x)
    assert np.all(y == 0.0)
    a = om.refined_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, 8, 2.0, y)
    b = oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, 8, 2.0)
    for k in ("pos", "opacity", "rgb", "idx"):
        np.testing.assert_allclose(a[k], b[k], atol=1e-15)


def test_fit_targets_inverts_refined_fan():
    g = scenes.gaussians(60, 8, 0.01, 0.1, flat=True)
    K = 8
    rng = np.random.default_rng(5)
    y = rng.normal(0, 0.1, (60, 3 * K + 4))
    y[:, 3 * K] = rng.uniform(-0.05, 0.05, 60) * np.asarray(g.opacity)   # keep the clamp inactive
    f = om.refined_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, K, 2.0, y)
    back = om.fit_targets(g.mean, g.scale, g.quat, g.opacity, g.rgb, K, 2.0, f)
    np.testing.assert_allclose(back, y, atol=1e-10)


def test_features_layout():
    g = scenes.gaussians(5, 9, 0.01, 0.1, flat=True)
    x = om.features(g.mean, g.scale, g.quat, g.opacity, g.rgb, 8)
    assert x.shape == (5, 15)
    np.testing.assert_allclose(x[:, 0:3], np.asarray(g.mean, np.float64).T)
    np.testing.assert_allclose(x[:, 3:6], np.asarray(g.scale, np.float64).T / 0.1)
    assert np.all(x[:, 6] >= 0) and np.allclose(np.linalg.norm(x[:, 6:10], axis=1), 1)
    assert np.all(x[:, 14] == 0.5)
