"""Pins of the oracle's smoothing-length iteration (a rule of this project, not
of the paper: the paper rebuilds its list each step with per-particle radii,
Sec. IV). The rule relies on n_i(h_i) being a non-decreasing step function of
h_i that depends on no other radius; the pins check that and that the rule
ends inside target +- tol."""
import numpy as np
import pytest

import oracle
from paper_2602_19873_amd import workloads


def test_count_is_monotone_in_own_radius_only():
    s = workloads.uniform_varied(3000, 61, target=30.0)
    base = s.h.copy()
    prev = None
    for f in (0.5, 0.8, 1.0, 1.3, 2.0):
        _, c = oracle.density(s.x, s.y, s.z, (base * f).astype(np.float32), None, "brute")
        if prev is not None:
            assert np.all(c >= prev)
        prev = c
    # changing other particles' radii does not change n_i
    h2 = base.copy()
    h2[1::2] *= 3.0
    _, c0 = oracle.density(s.x, s.y, s.z, base, None, "brute")
    _, c1 = oracle.density(s.x, s.y, s.z, h2, None, "brute")
    np.testing.assert_array_equal(c0[0::2], c1[0::2])


@pytest.mark.parametrize("kind", ["uniform", "sphere"])
def test_rule_converges(kind):
    if kind == "uniform":
        s = workloads.uniform_global(4000, 62, target=80.0)
        h0 = (s.h * 1.7).astype(np.float32)  # start far from the answer
        T = 40
    else:
        s = workloads.evrard_sphere(6000, 63, target=50.0)
        h0 = s.h
        T = 50
    h, rounds, unconv = oracle.h_iterate(s.x, s.y, s.z, h0, T, 1, 64, "grid")
    assert unconv == 0 and rounds <= 64
    _, c = oracle.density(s.x, s.y, s.z, h, None, "brute")
    assert np.all(np.abs(c - T) <= 1)


def test_zero_neighbours_doubles():
    x = np.array([0.0, 10.0], np.float32)
    z = np.zeros(2, np.float32)
    h, rounds, unconv = oracle.h_iterate(x, z, z, np.array([1.0, 1.0], np.float32), 1, 0, 3, "brute")
    # isolated particles keep doubling their radius until they see each other
    assert rounds == 3 and unconv == 2
    assert np.all(h == 8.0)


def _step(h, cnt, lo=0.0, hi=np.inf, target=100, tol=1):
    hn, l2, h2, mv = oracle.h_step(np.array([h]), np.array([cnt]), np.array([lo]), np.array([hi]), target, tol)
    return float(hn[0]), float(l2[0]), float(h2[0]), bool(mv[0])


def test_step_hand_values():
    """One round of the rule on hand-computed values: every branch."""
    # converged (|n - T| <= tol, both edges): nothing changes
    assert _step(1.0, 99) == (1.0, 0.0, np.inf, False)
    assert _step(1.0, 101, 0.5, 2.0) == (1.0, 0.5, 2.0, False)
    # no neighbours: the radius doubles, h becomes the lower bound
    assert _step(0.75, 0) == (1.5, 0.75, np.inf, True)
    # cube-root step inside the clamp: 2T neighbours -> h / 2^(1/3)
    hn, lo, hi, mv = _step(1.0, 200)
    assert abs(hn - 0.5 ** (1.0 / 3.0)) < 1e-15 and (lo, hi, mv) == (0.0, 1.0, True)
    # 8 / T of the neighbours: h (T / (T/8))^(1/3) = 2h exactly at the clamp
    hn, lo, hi, _ = _step(1.0, 100, target=800)
    assert hn == 2.0 and lo == 1.0
    # clamped from above (T/n = 100, cube root 4.64 -> 2) and below (0.1 -> 1/2)
    assert _step(1.0, 1)[0] == 2.0
    assert _step(1.0, 1000)[0] == 0.5
    # too many inside a bracket: hi = 1, the clamped 0.5 is not above lo = 0.9
    # -> midpoint 0.95
    hn, lo, hi, _ = _step(1.0, 1000, 0.9, 1.2)
    assert (hn, lo, hi) == (0.95, 0.9, 1.0)
    # too few inside a bracket: lo = 1, cube root 2^(1/3) = 1.26 not below
    # hi = 1.1 -> midpoint 1.05
    hn, lo, hi, _ = _step(1.0, 50, 0.5, 1.1)
    assert (hn, lo, hi) == (1.05, 1.0, 1.1)
    # upper side open: a proposal not above lo = 1.5 becomes 2 lo = 3
    hn, lo, hi, _ = _step(1.0, 50, 1.5, np.inf)
    assert (hn, lo, hi) == (3.0, 1.5, np.inf)
    # lower side open: a proposal not below hi = 0.4 becomes hi / 2 = 0.2
    hn, lo, hi, _ = _step(1.0, 1000, 0.0, 0.4)
    assert (hn, lo, hi) == (0.2, 0.0, 0.4)
    # a proposal exactly on a bracket end counts as outside: lo = 0.5, the
    # clamped step 0.5 -> midpoint of (0.5, 1.0)
    hn, lo, hi, _ = _step(1.0, 1000, 0.5, np.inf)
    assert (hn, lo, hi) == (0.75, 0.5, 1.0)


def test_two_rounds_on_a_hand_configuration():
    """Particle 0 at the origin; 2 neighbours at distance 1 (on the x axis)
    and 30 at distance 2.5 (the 6 axis points and the 24 points with
    coordinates a permutation of (1.5, 2, 0) up to signs). All coordinates are
    dyadic, so every FP32 distance is exact. Target 5, tol 0, start h = 2:
    round 1 sees 2 neighbours (lo = 2, h -> 2 (5/2)^(1/3) = 2.714); round 2
    sees 32 (hi = 2.714; the proposal 2.714 (5/32)^(1/3) = 1.46 lies within
    the clamp but not above lo, so h -> the midpoint (2 + 2.714) / 2)."""
    import itertools
    pts = {(0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (-1.0, 0.0, 0.0)}
    for a in range(3):
        for sgn in (-2.5, 2.5):
            v = [0.0, 0.0, 0.0]
            v[a] = sgn
            pts.add(tuple(v))
    for perm in itertools.permutations((1.5, 2.0, 0.0)):
        for sx, sy in itertools.product((-1.0, 1.0), repeat=2):
            signs = iter((sx, sy))
            pts.add(tuple(c * next(signs) if c else 0.0 for c in perm))
    p = np.array(sorted(pts, key=lambda t: (abs(t[0]) + abs(t[1]) + abs(t[2]), t)), np.float32)
    x, y, z = p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()
    n = len(p)
    d = np.sqrt(x.astype(np.float64) ** 2 + y.astype(np.float64) ** 2 + z.astype(np.float64) ** 2)
    assert d[0] == 0.0 and sorted(d[1:].tolist()) == [1.0] * 2 + [2.5] * 30
    h = np.full(n, 2.0, np.float32)
    _, cnt = oracle.density(x, y, z, h, None, "brute")
    assert cnt[0] == 2
    h1, lo, hi, _ = oracle.h_step(h, cnt, np.zeros(n), np.full(n, np.inf), 5, 0)
    assert abs(h1[0] - 2.0 * 2.5 ** (1.0 / 3.0)) < 1e-12 and lo[0] == 2.0 and hi[0] == np.inf
    h1 = h1.astype(np.float32)
    _, cnt = oracle.density(x, y, z, h1, None, "brute")
    assert cnt[0] == 32
    h2, lo, hi, _ = oracle.h_step(h1, cnt, lo, hi, 5, 0)
    assert lo[0] == 2.0 and hi[0] == float(h1[0])
    assert h2[0] == 0.5 * (2.0 + float(h1[0]))
