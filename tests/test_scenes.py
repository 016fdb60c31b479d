"""Host-side scene helpers (no GPU)."""
import numpy as np

from paper_2502_07754_amd import scenes


def test_permuted_stores_the_same_gaussians_in_the_given_order():
    g = scenes.gaussians(500, 3, 0.01, 0.1, flat=True, sh=True)
    order = np.random.default_rng(1).permutation(g.n)
    h = scenes.permuted(g, order)
    for name in ("mean", "scale", "quat", "rgb", "sh"):
        a, b = getattr(g, name), getattr(h, name)
        assert b.dtype == np.float32 and b.flags["C_CONTIGUOUS"]
        assert np.array_equal(b, a[:, order]), name
    assert np.array_equal(h.opacity, g.opacity[order])
    # the inverse order restores the scene bit for bit
    back = scenes.permuted(h, np.argsort(order))
    for name in ("mean", "scale", "quat", "opacity", "rgb", "sh"):
        assert np.array_equal(getattr(back, name), getattr(g, name)), name


def test_permuted_keeps_a_missing_sh_missing():
    g = scenes.gaussians(10, 0, 0.01, 0.1, flat=True)
    assert scenes.permuted(g, np.arange(10)[::-1]).sh is None
