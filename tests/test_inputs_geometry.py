"""Geometry generators standing in for the ones the paper names (Secs.
IV.B-C): the properties each construction guarantees (CPU)."""
import numpy as np
import pytest
from scipy import ndimage

from paper_1411_7051_amd import inputs


def test_tolerance_circles():
    rng = np.random.default_rng(1)
    cs = []
    m = inputs.tolerance_circles((200, 410), 0.4, (6.0, 20.0), 0.2, rng, centres=cs)
    f = m.mean()
    assert 0.4 <= f < 0.4 + np.pi * 20 ** 2 / m.size + 1e-9
    c = np.array(cs)
    for i in range(len(c)):
        dy = np.abs(c[i + 1:, 1] - c[i, 1])
        dy = np.minimum(dy, 200 - dy)
        d = np.hypot(c[i + 1:, 0] - c[i, 0], dy)
        assert np.all(d >= 0.8 * (c[i + 1:, 2] + c[i, 2]) - 1e-9)
    # no overlap at all with tol = 0
    cs0 = []
    inputs.tolerance_circles((100, 100), 0.2, (4.0, 8.0), 0.0, np.random.default_rng(2),
                             centres=cs0)
    c0 = np.array(cs0)
    d = np.hypot(*(c0[:, None, :2] - c0[None, :, :2]).transpose(2, 0, 1))
    r = c0[:, None, 2] + c0[None, :, 2]
    off = ~np.eye(len(c0), dtype=bool)
    dyw = np.abs(c0[:, None, 1] - c0[None, :, 1])
    dw = np.hypot(c0[:, None, 0] - c0[None, :, 0], np.minimum(dyw, 100 - dyw))
    assert np.all(dw[off] >= r[off] - 1e-9)


def test_qsgs_exact_fraction_and_mask():
    rng = np.random.default_rng(3)
    allowed = np.ones((120, 150), dtype=bool)
    allowed[:, :40] = False
    g = inputs.qsgs((120, 150), 0.3, rng, allowed=allowed)
    assert g.sum() == round(0.3 * g.size)
    assert not g[:, :40].any()
    a = inputs.qsgs((64, 64), 0.2, np.random.default_rng(7))
    b = inputs.qsgs((64, 64), 0.2, np.random.default_rng(7))
    assert np.array_equal(a, b)
    with pytest.raises(ValueError):
        inputs.qsgs((10, 10), 0.9, rng, allowed=allowed[:10, :10])


def test_qsgs_growth_is_clustered():
    """Growth from few cores gives far fewer, larger clusters than the same
    fraction of independent cells."""
    g = inputs.qsgs((128, 128), 0.3, np.random.default_rng(4), core=0.002)
    _, n_grown = ndimage.label(g)
    rnd = np.random.default_rng(4).random((128, 128)) < 0.3
    _, n_rand = ndimage.label(rnd)
    assert n_grown < n_rand / 5


def test_tree_fractures_percolate():
    f = inputs.tree_fractures((536, 1164), np.random.default_rng(6))
    lab, _ = ndimage.label(f)
    spanning = set(lab[:, 0][lab[:, 0] > 0]) & set(lab[:, -1][lab[:, -1] > 0])
    assert spanning
    assert 0.03 < f.mean() < 0.15


def test_trimodal_and_fractured_matrix():
    c = inputs.trimodal(seed=5)
    imp, perm, pore = (c.eps == 0), (c.eps == np.float32(0.5)), (c.eps == 1)
    assert abs(imp.mean() - 0.4) < 0.02 and perm.sum() == round(0.3 * c.nodes)
    assert np.all(np.isinf(c.k[pore])) and np.all(c.kn0[~perm] == 0)
    m = inputs.fractured_matrix(seed=6)
    assert m.shape == (536, 1164)
    frac = m.eps == 1
    assert 0.03 < frac.mean() < 0.15 and 0.08 < (m.eps == np.float32(0.2)).mean() < 0.11
