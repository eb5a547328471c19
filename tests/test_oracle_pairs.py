"""Pins of the oracle's pair set and cluster-pair list (Sec. II-A).

P = {(i, j): i != j, d2 < max(h_i, h_j)^2} under the fixed FP32 formula
d2 = fma(dz, dz, fma(dy, dy, dx*dx)). The cell-list search is checked against
O(N^2) brute force; both are checked against configurations whose neighbour
counts are known in closed form.
"""
import numpy as np
import pytest

import oracle
from paper_2602_19873_amd import workloads


def _mixed(n, seed, spread=3.0):
    rng = np.random.default_rng(seed)
    x, y, z = (rng.random(n).astype(np.float32) for _ in range(3))
    rc = workloads.radius_for_neighbours(n, 30.0)
    h = (rc * np.exp(rng.uniform(-np.log(spread), np.log(spread), n))).astype(np.float32)
    return x, y, z, h


def _lattice(k, a):
    g = np.arange(k, dtype=np.float32) * np.float32(a)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy()


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_grid_equals_brute_force(seed):
    x, y, z, h = _mixed(1500 + 37 * seed, seed)
    ob, nb = oracle.pairs_csr(x, y, z, h, "brute")
    og, ng = oracle.pairs_csr(x, y, z, h, "grid")
    np.testing.assert_array_equal(ob, og)
    np.testing.assert_array_equal(nb, ng)


def test_symmetric_and_irreflexive():
    x, y, z, h = _mixed(1200, 9, spread=5.0)
    offs, nbr = oracle.pairs_csr(x, y, z, h, "brute")
    pairs = set()
    for i in range(len(x)):
        for j in nbr[offs[i]:offs[i + 1]]:
            assert j != i
            pairs.add((i, int(j)))
    assert all((j, i) in pairs for (i, j) in pairs)


@pytest.mark.parametrize("h,count", [(0.13, 6), (0.18, 18), (0.22, 26), (0.125, 0)])
def test_lattice_counts(h, count):
    # simple cubic lattice of spacing 1/8 (exact in FP32): interior points see
    # 6 faces at a, 12 edges at sqrt(2) a, 8 corners at sqrt(3) a;
    # h = a exactly gives d2 == R2, which the strict test excludes
    a = 0.125
    x, y, z = _lattice(7, a)
    hh = np.full(x.shape, h, np.float32)
    offs, _ = oracle.pairs_csr(x, y, z, hh, "grid")
    deg = np.diff(offs)
    centre = 3 * 49 + 3 * 7 + 3
    assert deg[centre] == count


def test_coincident_and_max_radius():
    # coincident particles interact (d2 = 0 < R2); a small-radius particle is
    # a neighbour of a large-radius one and vice versa (R = max(h_i, h_j))
    x = np.array([0.0, 0.0, 0.3, 0.9], np.float32)
    y = np.zeros(4, np.float32)
    z = np.zeros(4, np.float32)
    h = np.array([0.01, 0.01, 0.5, 0.01], np.float32)
    offs, nbr = oracle.pairs_csr(x, y, z, h, "brute")
    got = {i: list(nbr[offs[i]:offs[i + 1]]) for i in range(4)}
    assert got == {0: [1, 2], 1: [0, 2], 2: [0, 1], 3: []}
    assert oracle.is_pair(0, 0, 0, 0.5, 0.5, 0, 0, 0.25) is False  # d == R exactly
    assert oracle.is_pair(0, 0, 0, 0.5, 0.4999, 0, 0, 0.25) is True


def _pairs_from_list(x, y, z, h, cs, offs, jj, mm):
    """Particle pairs recovered from the cluster list by filtering every
    (i-cluster, j-cluster) tile with the pair test."""
    n = len(x)
    got = set()
    for s in range(len(offs) - 1):
        for e in range(offs[s], offs[s + 1]):
            cj = int(jj[e])
            for c in range(64 // cs):
                if not (int(mm[e]) >> c) & 1:
                    continue
                for i in range(64 * s + c * cs, min(n, 64 * s + c * cs + cs)):
                    for j in range(cj * cs, min(n, cj * cs + cs)):
                        if i != j and oracle.is_pair(x[i], y[i], z[i], h[i], x[j], y[j], z[j], h[j]):
                            got.add((i, j))
    return got


@pytest.mark.parametrize("cs", [4, 8, 16])
def test_cluster_list_recovers_pair_set(cs):
    s = workloads.uniform_varied(700, 21, target=25.0)
    keys = oracle.hilbert_keys(s.x, s.y, s.z, s.box)
    p = oracle.sfc_order(keys)
    x, y, z, h = s.x[p], s.y[p], s.z[p], s.h[p]
    offs, jj, mm = oracle.cluster_list(x, y, z, h, cs, "brute")
    og, jg, mg = oracle.cluster_list(x, y, z, h, cs, "grid")
    np.testing.assert_array_equal(offs, og)
    np.testing.assert_array_equal(jj, jg)
    np.testing.assert_array_equal(mm, mg)
    # ascending, masks non-empty and within the super-cluster's i-clusters
    for sc in range(len(offs) - 1):
        seg = jj[offs[sc]:offs[sc + 1]]
        assert np.all(np.diff(seg.astype(np.int64)) > 0)
    assert np.all(mm > 0) and np.all(mm < (1 << (64 // cs)))
    po, pn = oracle.pairs_csr(x, y, z, h, "brute")
    ref = {(i, int(j)) for i in range(len(x)) for j in pn[po[i]:po[i + 1]]}
    assert _pairs_from_list(x, y, z, h, cs, offs, jj, mm) == ref


def test_cluster_list_masks_are_exact():
    # a mask bit is set iff some particle of that i-cluster has a pair in the
    # j-cluster (no bounding-box conservatism)
    s = workloads.uniform_global(600, 4, target=20.0)
    cs = 8
    x, y, z, h = s.x, s.y, s.z, s.h
    offs, jj, mm = oracle.cluster_list(x, y, z, h, cs, "brute")
    n = len(x)
    for sc in range(len(offs) - 1):
        for e in range(offs[sc], offs[sc + 1]):
            cj = int(jj[e])
            for c in range(8):
                ii = range(64 * sc + c * cs, min(n, 64 * sc + c * cs + cs))
                hit = any(i != j and oracle.is_pair(x[i], y[i], z[i], h[i], x[j], y[j], z[j], h[j])
                          for i in ii for j in range(cj * cs, min(n, cj * cs + cs)))
                assert hit == bool((int(mm[e]) >> c) & 1)


def test_cluster_level_symmetry():
    s = workloads.uniform_varied(1000, 8, target=40.0)
    cs = 8
    offs, jj, mm = oracle.cluster_list(s.x, s.y, s.z, s.h, cs, "grid")
    rel = set()
    for sc in range(len(offs) - 1):
        for e in range(offs[sc], offs[sc + 1]):
            for c in range(8):
                if (int(mm[e]) >> c) & 1:
                    rel.add((sc * 8 + c, int(jj[e])))
    assert all((cj, ci) in rel for (ci, cj) in rel)


def test_pair_set_independent_of_cluster_size():
    s = workloads.uniform_varied(520, 12, target=30.0)
    sets = []
    for cs in (4, 8, 16):
        offs, jj, mm = oracle.cluster_list(s.x, s.y, s.z, s.h, cs, "grid")
        sets.append(_pairs_from_list(s.x, s.y, s.z, s.h, cs, offs, jj, mm))
    assert sets[0] == sets[1] == sets[2]


def test_selected_super_clusters_match_full_list():
    s = workloads.uniform_varied(4096, 13, target=60.0)
    offs, jj, mm = oracle.cluster_list(s.x, s.y, s.z, s.h, 8, "grid")
    ids = np.array([0, 5, 17, 63])
    so, sj, sm = oracle.cluster_list(s.x, s.y, s.z, s.h, 8, "brute", sc_ids=ids)
    for k, sc in enumerate(ids):
        np.testing.assert_array_equal(sj[so[k]:so[k + 1]], jj[offs[sc]:offs[sc + 1]])
        np.testing.assert_array_equal(sm[so[k]:so[k + 1]], mm[offs[sc]:offs[sc + 1]])


def test_degenerate_sizes():
    for n in (0, 1, 7, 8, 9, 63, 64, 65):
        rng = np.random.default_rng(n)
        x, y, z = (rng.random(n).astype(np.float32) for _ in range(3))
        h = np.full(n, 2.0, np.float32)
        offs, jj, mm = oracle.cluster_list(x, y, z, h, 8, "grid")
        assert len(offs) == (n + 63) // 64 + 1
        if n >= 2:
            # every particle sees every other one: super-cluster 0 lists all clusters
            nc = (n + 7) // 8
            assert list(jj[offs[0]:offs[1]]) == list(range(nc))


@pytest.mark.parametrize("cs", [4, 8, 16])
def test_half_list_stores_each_pair_once(cs):
    """The half list (j > i) recovers exactly the upper half of P, its masks
    are exact for that half, and every entry is also in the full list with a
    mask that contains the half mask."""
    s = workloads.uniform_varied(700, 22, target=25.0)
    keys = oracle.hilbert_keys(s.x, s.y, s.z, s.box)
    p = oracle.sfc_order(keys)
    x, y, z, h = s.x[p], s.y[p], s.z[p], s.h[p]
    n = len(x)
    ho, hj, hm = oracle.cluster_list(x, y, z, h, cs, "brute", half=True)
    go, gj, gm = oracle.cluster_list(x, y, z, h, cs, "grid", half=True)
    np.testing.assert_array_equal(ho, go)
    np.testing.assert_array_equal(hj, gj)
    np.testing.assert_array_equal(hm, gm)
    po, pn = oracle.pairs_csr(x, y, z, h, "brute")
    upper = {(i, int(j)) for i in range(n) for j in pn[po[i]:po[i + 1]] if j > i}
    got = {(i, j) for (i, j) in _pairs_from_list(x, y, z, h, cs, ho, hj, hm) if j > i}
    assert got == upper
    # exact masks for the half: bit c iff some i of i-cluster c pairs with a
    # larger j of the j-cluster
    nsub = 64 // cs
    for sc in range(len(ho) - 1):
        for e in range(ho[sc], ho[sc + 1]):
            cj = int(hj[e])
            assert cj * cs + cs - 1 > 64 * sc  # never a j-cluster wholly before the super-cluster
            for c in range(nsub):
                ii = range(64 * sc + c * cs, min(n, 64 * sc + c * cs + cs))
                hit = any(j > i and oracle.is_pair(x[i], y[i], z[i], h[i], x[j], y[j], z[j], h[j])
                          for i in ii for j in range(cj * cs, min(n, cj * cs + cs)))
                assert hit == bool((int(hm[e]) >> c) & 1)
    fo, fj, fm = oracle.cluster_list(x, y, z, h, cs, "brute")
    for sc in range(len(ho) - 1):
        full = dict(zip(fj[fo[sc]:fo[sc + 1]].tolist(), fm[fo[sc]:fo[sc + 1]].tolist()))
        for e in range(ho[sc], ho[sc + 1]):
            fmask = full[int(hj[e])]
            assert (int(hm[e]) & ~fmask) == 0
    # about half the entries' pairs: the half list is the smaller one
    assert len(hj) < len(fj)
