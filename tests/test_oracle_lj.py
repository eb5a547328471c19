"""Pins of the oracle's Lennard-Jones 12/6 + Coulomb pass (Sec. III, the
Lennard-Jones benchmark: forces of the pairs inside an interaction cutoff).

The force formula is not retyped here. It is checked against facts the
potential fixes: the two-body minimum sits at 2^(1/6) sigma with depth -eps,
the Lennard-Jones energy vanishes at r = sigma, like charges repel with
k q q / r^2, every force is minus the gradient of the total energy (central
differences), the pair forces cancel in the sum (Newton's third law), and the
interacting pairs are exactly the FP32 pair set at radius r_cut."""
import math

import numpy as np
import pytest

import oracle


def _two(r, q=(0.0, 0.0)):
    x0 = np.float32(0.25)
    x1 = np.float32(0.25 + r)
    x = np.array([x0, x1], np.float32)
    o = np.full(2, 0.5, np.float32)
    return x, o, o.copy(), np.array(q, np.float32), float(x1) - float(x0)


def test_two_body_minimum_and_zero_crossing():
    x, y, z, q, r = _two(0.01)
    sigma = r * 2.0 ** (-1.0 / 6.0)
    out = oracle.lj(x, y, z, None, eps=1.5, sigma=sigma, r_cut=0.1)
    scale = 24.0 * 1.5 / r
    assert np.all(np.abs(out["f"]) <= 1e-12 * scale)
    np.testing.assert_allclose(out["e"], [-0.75, -0.75], rtol=1e-12)  # pair energy -eps, shared
    np.testing.assert_allclose(out["escale"], [0.75, 0.75], rtol=1e-12)
    assert list(out["nnb"]) == [1, 1]
    # at r = sigma the Lennard-Jones energy is zero and the force repulsive
    out = oracle.lj(x, y, z, None, eps=1.5, sigma=r, r_cut=0.1)
    assert np.all(np.abs(out["e"]) <= 1e-12)
    assert out["f"][0, 0] < 0.0 < out["f"][1, 0]


def test_coulomb_pair():
    for qa, qb in ((1.0, 1.0), (1.0, -2.0), (-0.5, -0.5)):
        x, y, z, q, r = _two(0.02, (qa, qb))
        out = oracle.lj(x, y, z, q, eps=0.0, sigma=1.0, coulomb=3.0, r_cut=0.1)
        mag = 3.0 * abs(qa * qb) / r ** 2
        np.testing.assert_allclose(abs(out["f"][0, 0]), mag, rtol=1e-12)
        # like charges push particle 0 (at smaller x) towards -x, unlike pull it towards +x
        assert (out["f"][0, 0] < 0) == (qa * qb > 0)
        np.testing.assert_allclose(out["f"][0], -out["f"][1], rtol=0, atol=1e-12 * mag)
        np.testing.assert_allclose(out["e"].sum(), 3.0 * qa * qb / r, rtol=1e-12)
        assert out["f"][0, 1] == 0.0 and out["f"][0, 2] == 0.0


def _cluster(n, seed, spread=0.02):
    rng = np.random.default_rng(seed)
    p = (0.5 + spread * rng.random((3, n))).astype(np.float32)
    q = rng.choice([-1.0, 1.0], n).astype(np.float32)
    return p[0], p[1], p[2], q


def test_force_is_minus_energy_gradient():
    # a jittered 3x2x2 lattice (spacing 0.005, no pair closer than 0.003),
    # every pair well inside the cutoff, so the total energy is smooth
    rng = np.random.default_rng(3)
    g = np.stack(np.meshgrid(np.arange(3), np.arange(2), np.arange(2), indexing="ij"), -1).reshape(-1, 3)
    p = (0.5 + 0.005 * (g + rng.uniform(-0.2, 0.2, g.shape))).astype(np.float32)
    x, y, z = (np.ascontiguousarray(p[:, a]) for a in range(3))
    q = rng.choice([-1.0, 1.0], 12).astype(np.float32)
    par = dict(eps=0.7, sigma=0.004, coulomb=2e-3, r_cut=0.5)
    out = oracle.lj(x, y, z, q, **par, method="brute")
    assert np.all(out["nnb"] == 11)
    d = np.float32(2.0 ** -22)  # exact shift of coordinates in [0.5, 1)
    for p in range(12):
        for ax, arr in enumerate((x, y, z)):
            lo, hi = arr.copy(), arr.copy()
            lo[p] -= d
            hi[p] += d
            args = [x, y, z]
            args[ax] = hi
            e_hi = oracle.lj(*args, q, **par, method="brute")["e"].sum()
            args[ax] = lo
            e_lo = oracle.lj(*args, q, **par, method="brute")["e"].sum()
            step = float(hi[p]) - float(lo[p])
            grad = (e_hi - e_lo) / step
            assert abs(-grad - out["f"][p, ax]) <= 1e-5 * out["scale"][p], (p, ax)


def test_newton_third_law_and_grid():
    rng = np.random.default_rng(8)
    n = 3000
    x, y, z = (rng.random(n).astype(np.float32) for _ in range(3))
    q = rng.choice([-1.0, 1.0], n).astype(np.float32)
    par = dict(eps=1.0, sigma=0.01, coulomb=1e-3, r_cut=0.06)
    g = oracle.lj(x, y, z, q, **par)
    b = oracle.lj(x, y, z, q, **par, method="brute")
    np.testing.assert_array_equal(g["nnb"], b["nnb"])
    np.testing.assert_allclose(g["f"], b["f"], rtol=1e-12, atol=1e-12 * g["scale"].max())
    np.testing.assert_allclose(g["e"], b["e"], rtol=1e-12, atol=1e-12)
    tot = g["f"].sum(axis=0)
    assert np.all(np.abs(tot) <= 1e-9 * g["scale"].sum())
    # the interacting pairs are the FP32 pair set at radius r_cut
    offs = oracle.pairs_csr(x, y, z, np.full(n, np.float32(0.06)), "grid")[0]
    np.testing.assert_array_equal(g["nnb"], np.diff(offs))


def test_rows_subset():
    x, y, z, q = _cluster(500, 5, spread=0.3)
    par = dict(eps=1.0, sigma=0.005, coulomb=1e-3, r_cut=0.05)
    full = oracle.lj(x, y, z, q, **par)
    idx = np.array([0, 17, 499, 250])
    sub = oracle.lj(x, y, z, q, **par, idx=idx)
    for k in ("f", "e", "scale", "escale", "nnb"):
        np.testing.assert_array_equal(sub[k], full[k][idx])


@pytest.mark.parametrize("n", [0, 1])
def test_degenerate(n):
    x = np.full(n, 0.5, np.float32)
    out = oracle.lj(x, x, x, None, r_cut=0.1)
    assert out["f"].shape == (n, 3) and np.all(out["f"] == 0.0) and np.all(out["nnb"] == 0)


def test_lattice_workload():
    # the benchmark recipe: ~200 neighbours inside the list radius and ~150
    # inside the interaction cutoff (interior atoms), neutral, no close pairs
    from paper_2602_19873_amd import workloads
    s = workloads.lj_lattice(24, 9)
    n = s.n
    assert n == 24 ** 3 and abs(float(s.q.sum())) == 0.0
    a = s.meta["spacing"]
    inner = np.all([(c > 0.25) & (c < 0.75) for c in (s.x, s.y, s.z)], axis=0)
    lst = oracle.lj(s.x, s.y, s.z, None, r_cut=s.meta["r_list"], idx=np.flatnonzero(inner))["nnb"]
    cut = oracle.lj(s.x, s.y, s.z, None, r_cut=s.meta["r_cut"], idx=np.flatnonzero(inner))["nnb"]
    assert 190 < lst.mean() < 210 and 142 < cut.mean() < 158
    offs, nbr = oracle.pairs_csr(s.x, s.y, s.z, np.full(n, np.float32(0.6 * a)), "grid")
    assert offs[-1] == 0  # no pair closer than (1 - 2 * 0.2) a
