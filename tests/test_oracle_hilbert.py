"""Pins of the oracle's Hilbert keys, stable order and clusters (Sec. II-A).

The paper only says the particles follow a Hilbert curve; which variant is
used does not change the pair set. The pins below are the properties that make
a curve a Hilbert curve: a bijection onto [0, 8^L), face-adjacent consecutive
cells, and keys whose 3-bit prefixes are the octree cells.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2602_19873_amd import workloads


def _cells(level):
    n = 1 << level
    return list(itertools.product(range(n), repeat=3))


@pytest.mark.parametrize("level", [1, 2, 3, 4, 5])
def test_bijection(level):
    keys = [oracle.hilbert3(x, y, z, level) for (x, y, z) in _cells(level)]
    assert sorted(keys) == list(range(8 ** level))


@pytest.mark.parametrize("level", [1, 2, 3, 4, 5])
def test_consecutive_cells_are_face_adjacent(level):
    cells = _cells(level)
    keys = [oracle.hilbert3(x, y, z, level) for (x, y, z) in cells]
    order = np.argsort(keys)
    pts = np.array(cells)[order]
    steps = np.abs(np.diff(pts, axis=0)).sum(axis=1)
    assert np.all(steps == 1)


@pytest.mark.parametrize("level", [2, 3, 4, 5])
def test_prefix_is_parent_cell(level):
    for (x, y, z) in _cells(level):
        k = oracle.hilbert3(x, y, z, level)
        assert k >> 3 == oracle.hilbert3(x >> 1, y >> 1, z >> 1, level - 1)


def test_level1_starts_at_origin_and_is_gray():
    keys = {oracle.hilbert3(x, y, z, 1): (x, y, z) for (x, y, z) in _cells(1)}
    assert keys[0] == (0, 0, 0)


def test_21bit_keys_nesting_random():
    rng = np.random.default_rng(5)
    for _ in range(2000):
        x, y, z = (int(v) for v in rng.integers(0, 2 ** 21, 3))
        k = oracle.hilbert3(x, y, z, 21)
        assert 0 <= k < 2 ** 63
        # the top 3L bits are the level-L cell's key
        L = int(rng.integers(1, 21))
        assert k >> (3 * (21 - L)) == oracle.hilbert3(x >> (21 - L), y >> (21 - L), z >> (21 - L), L)


def test_quantisation_endpoints():
    box = (0.0, 1.0, 0.0, 1.0, 0.0, 1.0)
    x = np.array([0.0, 0.5, np.nextafter(np.float32(1.0), np.float32(0.0)), 1.0, -0.25, 7.0], np.float32)
    keys = oracle.hilbert_keys(x, np.zeros_like(x), np.zeros_like(x), box)
    q = [0, 2 ** 20, 2 ** 21 - 1, 2 ** 21 - 1, 0, 2 ** 21 - 1]
    for k, qx in zip(keys, q):
        assert int(k) == oracle.hilbert3(qx, 0, 0, 21)


def test_stable_order_invariants():
    rng = np.random.default_rng(11)
    # many ties: positions on a coarse lattice
    x = (rng.integers(0, 4, 5000) / 4.0).astype(np.float32)
    y = (rng.integers(0, 4, 5000) / 4.0).astype(np.float32)
    z = (rng.integers(0, 4, 5000) / 4.0).astype(np.float32)
    keys = oracle.hilbert_keys(x, y, z, workloads.UNIT_BOX)
    perm = oracle.sfc_order(keys).astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(5000))
    sk = keys[perm]
    assert np.all(sk[1:] >= sk[:-1])
    ties = sk[1:] == sk[:-1]
    assert np.all(perm[1:][ties] > perm[:-1][ties])


def test_sfc_order_is_spatially_local():
    # consecutive particles along the curve are close on average (Sec. II-A)
    s = workloads.uniform_global(32768, 3)
    keys = oracle.hilbert_keys(s.x, s.y, s.z, s.box)
    p = oracle.sfc_order(keys)
    xs, ys, zs = s.x[p], s.y[p], s.z[p]
    step = np.sqrt(np.diff(xs) ** 2 + np.diff(ys) ** 2 + np.diff(zs) ** 2)
    spacing = (1.0 / 32768) ** (1.0 / 3.0)
    assert np.median(step) < 1.5 * spacing
    r = np.random.default_rng(0).permutation(32768)
    rstep = np.sqrt(np.diff(s.x[r]) ** 2 + np.diff(s.y[r]) ** 2 + np.diff(s.z[r]) ** 2)
    assert np.median(step) < 0.05 * np.median(rstep)


def test_cluster_bboxes_tight():
    rng = np.random.default_rng(2)
    n = 203
    x, y, z = (rng.random(n).astype(np.float32) for _ in range(3))
    h = rng.random(n).astype(np.float32)
    for cs in (4, 8, 16):
        bb = oracle.cluster_bboxes(x, y, z, h, cs)
        assert bb.shape == ((n + cs - 1) // cs, 8)
        for c in range(bb.shape[0]):
            idx = np.arange(c * cs, min(n, c * cs + cs))
            for a, arr in enumerate((x, y, z)):
                assert np.all(arr[idx] >= bb[c, a]) and np.all(arr[idx] <= bb[c, 4 + a])
                assert bb[c, a] in arr[idx] and bb[c, 4 + a] in arr[idx]
            assert bb[c, 3] == h[idx].max()
