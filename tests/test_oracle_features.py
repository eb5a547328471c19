"""Pins of the oracle's seed features (the learned h-seed is this library's
addition, not the paper's).

The key-cell occupancy features are checked against a count of particles in
the same cube cell of the level's grid, found from integer cell coordinates
(no keys): a Hilbert-key prefix of L digits names exactly one such cell, so
the two counts agree only if the prefix search is right. The box features are
checked against boxes computed here directly."""
import math

import numpy as np

import oracle


def _system(n, seed):
    rng = np.random.default_rng(seed)
    # clumpy: half uniform, half in a small ball, so occupancies vary widely
    u = rng.random((n // 2, 3))
    c = 0.5 + 0.05 * rng.standard_normal((n - n // 2, 3))
    p = np.clip(np.concatenate([u, c]), 0.0, 0.999).astype(np.float32)
    h = (0.03 * np.exp(rng.uniform(-1.5, 1.5, n))).astype(np.float32)
    return p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy(), h


def _sorted(n, seed):
    x, y, z, h = _system(n, seed)
    box = (0.0, 1.0, 0.0, 1.0, 0.0, 1.0)
    keys = oracle.hilbert_keys(x, y, z, box)
    o = np.argsort(keys, kind="stable")
    return keys[o], x[o], y[o], z[o], h[o]


def _boxes(x, y, z, h):
    n = x.shape[0]
    nc = (n + 7) // 8
    bb = np.zeros((nc, 8), dtype=np.float32)
    for c in range(nc):
        s = slice(8 * c, min(n, 8 * c + 8))
        bb[c] = [x[s].min(), y[s].min(), z[s].min(), h[s].max(), x[s].max(), y[s].max(), z[s].max(), 0.0]
    return bb


def test_occupancy_is_the_cube_cell_count():
    keys, x, y, z, h = _sorted(4000, 5)
    bb = _boxes(x, y, z, h)
    T = 100
    f = oracle.hseed_features(keys, h, np.full(x.shape[0], 40), bb, 1.0, T)
    # integer cell coordinates on the 2^21 grid (unit box: scale 2^21)
    q = [np.minimum((a.astype(np.float32) * np.float32(2 ** 21)).astype(np.int64), 2 ** 21 - 1) for a in (x, y, z)]
    lev = np.log2(1.0 / h.astype(np.float64))
    L0 = np.clip(np.rint(lev), 2, 20).astype(np.int64)
    for d in (-1, 0, 1):
        occ = np.empty(x.shape[0])
        for i in range(x.shape[0]):
            L = L0[i] + d
            sh = 21 - L
            same = ((q[0] >> sh) == (q[0][i] >> sh)) & ((q[1] >> sh) == (q[1][i] >> sh)) & \
                   ((q[2] >> sh) == (q[2][i] >> sh))
            occ[i] = same.sum()
        np.testing.assert_allclose(f[:, 4 + d], np.log(1.0 + occ) - math.log(T), rtol=0, atol=1e-12)
    np.testing.assert_allclose(f[:, 6], lev - L0, atol=1e-12)
    inner = (L0 > 2) & (L0 < 20)
    assert inner.any() and np.all(np.abs(f[inner, 6]) <= 0.5 + 1e-12)
    np.testing.assert_allclose(f[:, 7], 0.0, atol=1e-15)


def test_count_and_box_features():
    keys, x, y, z, h = _sorted(1000, 6)
    bb = _boxes(x, y, z, h)
    n = x.shape[0]
    nnb = np.arange(n) % 300
    T = 150
    f = oracle.hseed_features(keys, h, nnb, bb, 1.0, T)
    np.testing.assert_allclose(f[:, 0], np.log((nnb + 1.0) / T), atol=1e-12)
    np.testing.assert_allclose(f[:, 7], math.log(1.5), atol=1e-12)
    for i in (0, 7, 8, 500, n - 1):
        c = i // 8
        diag = math.sqrt(sum((float(bb[c, 4 + a]) - float(bb[c, a])) ** 2 for a in range(3)))
        assert abs(f[i, 1] - math.log(max(diag / float(h[i]), 1e-3))) < 1e-12
        s0 = (i // 64) * 64
        s = slice(s0, min(n, s0 + 64))
        sd = math.sqrt((float(x[s].max()) - float(x[s].min())) ** 2 + (float(y[s].max()) - float(y[s].min())) ** 2 +
                       (float(z[s].max()) - float(z[s].min())) ** 2)
        assert abs(f[i, 2] - math.log(max(sd / float(h[i]), 1e-3))) < 1e-12
    # no count yet (the seed before the first round): feature 0 is zero, the
    # rest unchanged
    g = oracle.hseed_features(keys, h, None, bb, 1.0, T)
    assert np.all(g[:, 0] == 0.0)
    np.testing.assert_array_equal(g[:, 1:], f[:, 1:])
