"""Pins of the oracle's periodic boundaries (Sec. II-A: periodic distances
computed per pair, no shift vectors).

On coordinates and radii that are multiples of 2^-10 in a box of period 1,
every FP32 step of the minimum-image pair formula is exact, so the pair set
must equal an integer brute force over all 27 images and be invariant under
periodic translations. Lattices that fill the periodic box give every
particle the same neighbours (6 / 18 / 26 shells), the same density and zero
Lennard-Jones force."""
import numpy as np
import pytest

import oracle

Q = 1024  # grid of 2^-10


def _dyadic(n, seed, rlo=40, rhi=90):
    rng = np.random.default_rng(seed)
    ip = rng.integers(0, Q, (3, n))
    ir = rng.integers(rlo, rhi, n)
    p = (ip / Q).astype(np.float32)
    return ip, ir, p[0], p[1], p[2], (ir / Q).astype(np.float32)


def _brute_int(ip, ir, periodic):
    """Pairs by integer arithmetic: squared minimum-image distance < max(R)^2."""
    n = ip.shape[1]
    d2 = np.zeros((n, n), np.int64)
    for a in range(3):
        d = ip[a][None, :] - ip[a][:, None]
        if periodic[a]:
            d = np.minimum(np.abs(d), Q - np.abs(d))
        d2 += d * d
    r = np.maximum(ir[None, :], ir[:, None])
    adj = d2 < r * r
    np.fill_diagonal(adj, False)
    return adj


def _adj(offs, nbr, n):
    a = np.zeros((n, n), bool)
    for i in range(n):
        a[i, nbr[offs[i]:offs[i + 1]]] = True
    return a


@pytest.mark.parametrize("periodic", [(1, 1, 1), (1, 0, 1), (0, 0, 0)])
@pytest.mark.parametrize("method", ["brute", "grid"])
def test_dyadic_pairs_equal_integer_images(periodic, method):
    ip, ir, x, y, z, h = _dyadic(500, 3)
    per = [1.0 if p else 0.0 for p in periodic]
    offs, nbr = oracle.pairs_csr(x, y, z, h, method, period=per)
    ref = _brute_int(ip, ir, periodic)
    np.testing.assert_array_equal(_adj(offs, nbr, 500), ref)
    if any(periodic):
        # wrapping pairs exist, so the test sees the minimum image at work
        assert ref.sum() > _brute_int(ip, ir, (0, 0, 0)).sum()


def test_translation_invariance():
    ip, ir, x, y, z, h = _dyadic(400, 4)
    per = [1.0, 1.0, 1.0]
    offs, nbr = oracle.pairs_csr(x, y, z, h, "grid", period=per)
    base = _adj(offs, nbr, 400)
    for shift in ((300, 0, 0), (17, 900, 512), (1023, 1, 640)):
        sp = [((ip[a] + shift[a]) % Q / Q).astype(np.float32) for a in range(3)]
        o2, n2 = oracle.pairs_csr(*sp, h, "grid", period=per)
        np.testing.assert_array_equal(_adj(o2, n2, 400), base)


def _lattice(k):
    g = (np.indices((k, k, k)).reshape(3, -1) + 0.5) / k
    return [a.astype(np.float32) for a in g]


@pytest.mark.parametrize("k", [5, 8])
def test_lattice_shells(k):
    x, y, z = _lattice(k)
    a = 1.0 / k
    for r, want in ((1.01 * a, 6), (1.5 * a, 18), (1.8 * a, 26)):
        h = np.full(x.shape[0], r, np.float32)
        offs, _ = oracle.pairs_csr(x, y, z, h, "grid", period=[1, 1, 1])
        assert np.all(np.diff(offs) == want)
        rho, nnb = oracle.density(x, y, z, h, period=[1, 1, 1])
        assert np.all(nnb == want)
        # k = 8 puts the sites on multiples of 2^-4 (exact in FP32); k = 5 rounds
        # them, which moves the densities by ~1e-9 relative
        assert np.ptp(rho) <= (1e-12 if k == 8 else 1e-6) * rho.max()
    # open boundaries: corner particles see fewer
    offs, _ = oracle.pairs_csr(x, y, z, np.full(x.shape[0], 1.01 * a, np.float32), "grid")
    assert np.diff(offs).min() == 3


def test_tiny_periodic_box_grid_equals_brute():
    # radii close to half the period: one or two cells per axis, so the wrapped
    # stencil must not visit a cell twice
    ip, ir, x, y, z, h = _dyadic(300, 5, rlo=300, rhi=500)
    per = [1.0, 1.0, 1.0]
    ob, nb = oracle.pairs_csr(x, y, z, h, "brute", period=per)
    og, ng = oracle.pairs_csr(x, y, z, h, "grid", period=per)
    np.testing.assert_array_equal(ob, og)
    np.testing.assert_array_equal(nb, ng)
    np.testing.assert_array_equal(_adj(ob, nb, 300), _brute_int(ip, ir, (1, 1, 1)))


def test_long_period_is_open():
    rng = np.random.default_rng(6)
    x, y, z = (rng.random(2000).astype(np.float32) for _ in range(3))
    h = (0.03 * rng.uniform(0.5, 1.5, 2000)).astype(np.float32)
    o0, n0 = oracle.pairs_csr(x, y, z, h, "grid")
    o1, n1 = oracle.pairs_csr(x, y, z, h, "grid", period=[4.0, 0.0, 4.0])
    np.testing.assert_array_equal(o0, o1)
    np.testing.assert_array_equal(n0, n1)


@pytest.mark.parametrize("cs,half", [(8, False), (8, True), (4, False), (16, True)])
def test_cluster_list_recovers_periodic_pairs(cs, half):
    rng = np.random.default_rng(7)
    n = 1500
    x, y, z = (rng.random(n).astype(np.float32) for _ in range(3))
    h = (0.07 * rng.uniform(0.6, 1.4, n)).astype(np.float32)
    per = [1.0, 1.0, 0.0]
    keys = oracle.hilbert_keys(x, y, z, (0, 1, 0, 1, 0, 1))
    o = oracle.sfc_order(keys)
    x, y, z, h = x[o], y[o], z[o], h[o]
    offs, nbr = oracle.pairs_csr(x, y, z, h, "grid", period=per)
    lo, lj, lm = oracle.cluster_list(x, y, z, h, cs, half=half, period=per)
    lb, jb, mb = oracle.cluster_list(x, y, z, h, cs, method="brute", half=half, period=per)
    np.testing.assert_array_equal(lo, lb)
    np.testing.assert_array_equal(lj, jb)
    np.testing.assert_array_equal(lm, mb)
    got = set()
    for s in range(len(lo) - 1):
        for e in range(lo[s], lo[s + 1]):
            for c in range(64 // cs):
                if (lm[e] >> c) & 1:
                    for i in range(64 * s + c * cs, min(n, 64 * s + c * cs + cs)):
                        for j in range(int(lj[e]) * cs, min(n, int(lj[e]) * cs + cs)):
                            if i != j and (not half or j > i):
                                got.add((i, j))
    want = set()
    for i in range(n):
        for j in nbr[offs[i]:offs[i + 1]]:
            if not half or j > i:
                want.add((i, int(j)))
    # every pair of P is covered by a listed tile, and every listed tile holds a pair
    assert want <= got
    pairs_by_tile = {}
    for (i, j) in want:
        pairs_by_tile[(i // cs, j // cs)] = True
    for s in range(len(lo) - 1):
        for e in range(lo[s], lo[s + 1]):
            for c in range(64 // cs):
                if (lm[e] >> c) & 1:
                    assert ((64 * s) // cs + c, int(lj[e])) in pairs_by_tile


def test_lj_periodic_lattice_and_momentum():
    x, y, z = _lattice(8)
    a = 1.0 / 8
    q = np.where((np.indices((8, 8, 8)).reshape(3, -1).sum(0) % 2) == 0, 0.5, -0.5).astype(np.float32)
    par = dict(eps=1.0, sigma=0.9 * a, coulomb=4 * a, r_cut=2.2 * a, period=[1, 1, 1])
    out = oracle.lj(x, y, z, q, **par)
    assert np.all(np.abs(out["f"]) <= 1e-10 * out["scale"][:, None])  # perfect lattice: forces cancel
    assert np.ptp(out["e"]) <= 1e-12 * np.abs(out["e"]).max()
    rng = np.random.default_rng(8)
    xj, yj, zj = ((c + rng.uniform(-0.2, 0.2, c.shape) * a) % 1.0 for c in (x, y, z))
    xj, yj, zj = (np.float32(v) for v in (xj, yj, zj))
    g = oracle.lj(xj, yj, zj, q, **par)
    b = oracle.lj(xj, yj, zj, q, **par, method="brute")
    np.testing.assert_allclose(g["f"], b["f"], rtol=1e-12, atol=1e-12 * g["scale"].max())
    assert np.all(np.abs(g["f"].sum(axis=0)) <= 1e-9 * g["scale"].sum())
