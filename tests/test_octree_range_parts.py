"""The node-box range query of the octree in closed form: the units a node's
particle range [first, end) leaves at each level (level 0: particles; level
l >= 1: boxes of cs * 8^(l-1) particles) are the whole units of
[ceil(first / 2^sh), floor(end / 2^sh)) whose next-level unit is not whole
inside the range (all of them on the coarsest level). The node-box kernel
splits every (level, end) part over 16 lanes from this formula; here the
parts are checked against the walk that takes ragged items level by level,
and shown to cover the range exactly once."""
import random

import pytest


def walk(first, end, cshift, nlvl):
    """Ragged particles at both ends, then whole groups coarsening one level
    at a time; the last box level takes what is left."""
    items = set()
    a, b = first, end
    cm = (1 << cshift) - 1
    while a < b and (a & cm):
        items.add((0, a))
        a += 1
    while b > a and (b & cm):
        b -= 1
        items.add((0, b))
    a >>= cshift
    b >>= cshift
    for l in range(nlvl):
        if not a < b:
            break
        last = l + 1 == nlvl
        while a < b and (last or (a & 7)):
            items.add((l + 1, a))
            a += 1
        while b > a and (last or (b & 7)):
            b -= 1
            items.add((l + 1, b))
        a >>= 3
        b >>= 3
    return items


def parts(first, end, cshift, nlvl, lanes=16):
    """The kernel's closed form: lane q takes parts q, q + lanes, ... (part
    2l + e: level l, end e), loading four items at a time from a clamped
    index (repeats do not change a union of boxes)."""
    items = set()
    for q in range(lanes):
        for part in range(q, 2 * (nlvl + 1), lanes):
            l = part >> 1
            sh = 0 if l == 0 else cshift + 3 * (l - 1)
            lo = (first + (1 << sh) - 1) >> sh
            hi = end >> sh
            if lo >= hi:
                continue
            if l == nlvl:
                i0, i1 = lo, (lo if part & 1 else hi)
            else:
                m = (1 << cshift) - 1 if l == 0 else 7
                f = min((lo + m) & ~m, hi)
                bk = max(hi & ~m, f)
                i0, i1 = (bk, hi) if part & 1 else (lo, f)
            for t0 in range(i0, i1, 4):
                for u in range(4):
                    items.add((l, min(t0 + u, i1 - 1)))
    return items


def levels(n, cshift):
    m = (n + (1 << cshift) - 1) >> cshift
    nl = 0
    while m > 1 and nl < 12:
        m = (m + 7) // 8
        nl += 1
    return nl + 1


@pytest.mark.parametrize("cshift", [2, 3, 4])
def test_parts_match_the_walk_and_tile_the_range(cshift):
    rng = random.Random(1000 + cshift)
    for _ in range(4000):
        n = rng.choice([1, 5, 17, 100, 1000, 4099, 100000, 1 << 21])
        nlvl = levels(n, cshift)
        first = rng.randrange(n)
        end = rng.randrange(first + 1, n + 1) if rng.random() < 0.7 else min(n, first + rng.randrange(1, 300))
        got = parts(first, end, cshift, nlvl)
        assert got == walk(first, end, cshift, nlvl), (first, end, cshift, nlvl)
        # every item lies in the range and the items cover it exactly once
        spans = sorted((t << (0 if l == 0 else cshift + 3 * (l - 1)), (t + 1) << (0 if l == 0 else cshift + 3 * (l - 1)))
                       for l, t in got)
        pos = first
        for lo, hi in spans:
            assert lo == pos
            pos = hi
        assert pos == end
