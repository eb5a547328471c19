"""Pins of the oracle's FP32 pair formula on inputs where rounding matters.

The pair set (the neighbour criterion with per-particle radii, Sec. II-A,
taken symmetric as max(h_i, h_j)) is defined by one FP32 sequence:
dx = f32(x_j - x_i) (likewise dy, dz; on a periodic axis the rounded
difference moves by one period when it exceeds f32(L/2) in magnitude, the
shift rounded again), d2 = fma(dz, dz, fma(dy, dy, f32(dx * dx))) with each
fused step rounded once, and (i, j) is a pair iff d2 < f32(R * R) with
R = max(h_i, h_j). The own-radius count uses R = h_i.

Here that sequence is evaluated in exact rational arithmetic, rounding to the
nearest binary32 (ties to even) after every step, independently of the
oracle's C code. Pairs are drawn so that d2 sits at the radius: the radius is
chosen between the stated formula's d2 and the d2 of a plausible wrong
formula (plain sums, the reversed fused order, one final rounding, an
unrounded difference or an unrounded radius square). The oracle must follow
the stated formula on every pair, and each wrong formula must be contradicted
by some pair, so a slip in the oracle's rounding order cannot pass.
"""
import math
from fractions import Fraction as F

import numpy as np

import oracle


def f32r(q: F) -> F:
    """q rounded to the nearest binary32 value, ties to even (subnormals
    included; no input here comes near overflow)."""
    if q == 0:
        return F(0)
    sign = -1 if q < 0 else 1
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while F(2) ** e > a:
        e -= 1
    while F(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -126)
    quantum = F(2) ** (e - 23)
    m = a / quantum
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > F(1, 2) or (rem == F(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * fl * quantum


def fr(v) -> F:
    return F(float(np.float32(v)))


def as_f32(q: F) -> np.float32:
    v = np.float32(float(q))
    assert F(float(v)) == q, "not a binary32 value"
    return v


def _diff(xj, xi, L=None):
    d = f32r(fr(xj) - fr(xi))
    if L is not None:
        hl = f32r(fr(L) / 2)
        if d > hl:
            d = f32r(d - fr(L))
        elif d < -hl:
            d = f32r(d + fr(L))
    return d


def d2_stated(pi, pj, L=None):
    dx, dy, dz = (_diff(pj[a], pi[a], L) for a in range(3))
    dxx = f32r(dx * dx)
    t = f32r(dy * dy + dxx)
    return f32r(dz * dz + t)


def d2_plain_sum(pi, pj):
    dx, dy, dz = (_diff(pj[a], pi[a]) for a in range(3))
    s = f32r(f32r(dx * dx) + f32r(dy * dy))
    return f32r(s + f32r(dz * dz))


def d2_reversed(pi, pj):
    dx, dy, dz = (_diff(pj[a], pi[a]) for a in range(3))
    t = f32r(dy * dy + f32r(dz * dz))
    return f32r(dx * dx + t)


def d2_one_rounding(pi, pj):
    dx, dy, dz = (_diff(pj[a], pi[a]) for a in range(3))
    return f32r(dx * dx + dy * dy + dz * dz)


def d2_exact_diff(pi, pj):
    dx, dy, dz = (fr(pj[a]) - fr(pi[a]) for a in range(3))
    t = f32r(dy * dy + f32r(dx * dx))
    return f32r(dz * dz + t)


WRONG = {"plain_sum": d2_plain_sum, "reversed_fma": d2_reversed, "one_rounding": d2_one_rounding,
         "exact_diff": d2_exact_diff}


def _radius_between(lo: F, hi: F):
    """A binary32 R with lo < f32(R * R) <= hi, or None."""
    r0 = np.float32(math.sqrt(float(hi)))
    cand = [r0]
    up = dn = r0
    for _ in range(4):
        up = np.nextafter(up, np.float32(np.inf), dtype=np.float32)
        dn = np.nextafter(dn, np.float32(0.0), dtype=np.float32)
        cand += [up, dn]
    for r in cand:
        r2 = f32r(fr(r) * fr(r))
        if lo < r2 <= hi:
            return r
    return None


def _draw_cases(seed, count):
    """Pairs whose radius separates the stated d2 from a wrong formula's."""
    rng = np.random.default_rng(seed)
    cases = []
    for _ in range(count):
        # coordinates spread over magnitudes, so that differences of
        # coordinates far from each other in size are inexact
        pi = (rng.random(3) * 10.0 ** rng.uniform(-2, 0, 3)).astype(np.float32)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        dist = 10.0 ** rng.uniform(-3, -0.7)
        pj = (pi.astype(np.float64) + dist * u).astype(np.float32)
        a = d2_stated(pi, pj)
        name = list(WRONG)[rng.integers(len(WRONG))]
        b = WRONG[name](pi, pj)
        if a == b:
            continue
        r = _radius_between(min(a, b), max(a, b))
        if r is None:
            continue
        other = np.float32(float(r) * rng.uniform(0.3, 0.99))
        hi, hj = (r, other) if rng.random() < 0.5 else (other, r)
        cases.append((pi, pj, hi, hj, name, a < f32r(fr(r) * fr(r)), b < f32r(fr(r) * fr(r))))
    return cases


def test_f32r_matches_numpy_rounding():
    # the rational rounding agrees with the hardware's float32 arithmetic
    rng = np.random.default_rng(5)
    for _ in range(2000):
        a, b = rng.random(2).astype(np.float32) * np.float32(10.0 ** rng.integers(-3, 3))
        assert f32r(fr(a) * fr(b)) == fr(np.float32(a * b))
        assert f32r(fr(a) - fr(b)) == fr(np.float32(a - b))
    # ties to even: 1 + 2^-24 rounds to 1, 1 + 3 * 2^-24 rounds to 1 + 2^-22
    assert f32r(1 + F(1, 2 ** 24)) == 1
    assert f32r(1 + F(3, 2 ** 24)) == 1 + F(1, 2 ** 22)
    assert f32r(F(1, 2 ** 150) * 3) == F(1, 2 ** 149) * 2  # subnormal tie -> even


def test_pair_formula_on_rounding_sensitive_pairs():
    cases = _draw_cases(20260219, 6000)
    assert len(cases) > 300
    hit = {k: 0 for k in WRONG}
    for pi, pj, hi, hj, name, stated, wrong in cases:
        got = oracle.is_pair(pi[0], pi[1], pi[2], hi, pj[0], pj[1], pj[2], hj)
        assert got == stated, (pi, pj, hi, hj)
        # P is symmetric: the swapped pair gives the bitwise-negated
        # differences and the same max radius
        assert oracle.is_pair(pj[0], pj[1], pj[2], hj, pi[0], pi[1], pi[2], hi) == stated
        assert wrong != stated
        hit[name] += 1
    # every wrong formula is contradicted by many pairs
    assert min(hit.values()) >= 20, hit


def test_own_radius_count_on_rounding_sensitive_pairs():
    """The neighbour count n_i (own radius h_i) uses the same sequence: a
    two-particle system gives particle 0 a neighbour iff d2 < f32(h_0^2)."""
    cases = _draw_cases(20260220, 3000)[:200]
    x = np.zeros(2, np.float32)
    y = np.zeros(2, np.float32)
    z = np.zeros(2, np.float32)
    for pi, pj, hi, hj, name, stated, wrong in cases:
        r = max(hi, hj)
        x[:], y[:], z[:] = (pi[0], pj[0]), (pi[1], pj[1]), (pi[2], pj[2])
        h = np.array([r, np.float32(1e-6)], np.float32)
        _, cnt = oracle.density(x, y, z, h, None, "brute")
        assert cnt[0] == (1 if stated else 0) and cnt[1] == 0


def test_radius_square_is_rounded():
    """(i, j) with d2 equal to f32(R^2) where f32(R^2) < R^2: the rounded
    square excludes the pair, an unrounded one would include it."""
    rng = np.random.default_rng(11)
    found = 0
    for _ in range(4000):
        r = np.float32(rng.uniform(0.01, 0.2))
        r2 = f32r(fr(r) * fr(r))
        if not r2 < fr(r) * fr(r):
            continue
        # a pair along x whose d2 = f32(dx * dx) equals r2
        xi = np.float32(rng.uniform(0.3, 0.6))
        xj = np.float32(float(xi) + float(r))
        d = _diff(xj, xi)
        if f32r(d * d) != r2:
            continue
        zero = np.float32(0.0)
        assert not oracle.is_pair(xi, zero, zero, r, xj, zero, zero, np.float32(0.001))
        found += 1
    assert found > 20


def test_periodic_image_rounding():
    """On a periodic axis the oracle shifts the rounded difference by one
    period and rounds again (the stated sequence); pairs across the face are
    drawn at the radius as above."""
    rng = np.random.default_rng(13)
    L = np.float32(1.0)
    checked = 0
    for _ in range(3000):
        pi = rng.random(3).astype(np.float32)
        pi[0] = np.float32(rng.uniform(0.0, 0.02))
        pj = (pi.astype(np.float64) + rng.normal(size=3) * 0.01).astype(np.float32)
        pj[0] = np.float32(1.0 - rng.uniform(0.0, 0.02))
        a = d2_stated(pi, pj, L)
        # the image taken on the exact difference, rounded once
        dx = f32r(fr(pj[0]) - fr(pi[0]) - fr(L))
        dy, dz = _diff(pj[1], pi[1]), _diff(pj[2], pi[2])
        b = f32r(dz * dz + f32r(dy * dy + f32r(dx * dx)))
        lo, hi = (min(a, b), max(a, b)) if a != b else (a - a / 2 ** 20, a)
        r = _radius_between(lo, hi)
        if r is None:
            continue
        x, y, z = (np.array([pi[k], pj[k]], np.float32) for k in range(3))
        h = np.array([r, r], np.float32)
        offs, nbr = oracle.pairs_csr(x, y, z, h, "brute", period=(L, L, L))
        got = int(offs[1] - offs[0]) == 1
        assert got == (a < f32r(fr(r) * fr(r))), (pi, pj, r)
        checked += 1
    assert checked > 500
