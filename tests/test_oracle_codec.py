"""Pins of the oracle's nibble encoding (Sec. II-B, Tables I and II; Sec. II-C)."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table1_rows():
    rows = []
    with open(os.path.join(GOLDEN, "table1_encoding.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            diffs, mask, info, data = (s.strip() for s in line.split("|"))
            rows.append(([int(v) for v in diffs.split(",")], mask,
                         "" if info == "-" else info, "" if data == "-" else data))
    return rows


@pytest.mark.parametrize("row", _table1_rows(), ids=lambda r: r[1])
def test_table1_rows(row):
    diffs, mask, info, data = row
    bits, inf, dat = oracle.block_symbols(diffs)
    assert "".join(str(int(b)) for b in bits) == mask
    assert "".join("%X" % v for v in inf) == info
    assert "".join("%X" % v for v in dat) == data


def _table2_rows():
    rows = []
    with open(os.path.join(GOLDEN, "table2_bits.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rng, bits = line.split("|")
            lo, hi = (int(v) for v in rng.split())
            rows.append((lo, hi, int(bits)))
    return rows


def _cost_bits(v):
    bits, inf, dat = oracle.block_symbols([v])
    return len(bits) + 4 * len(inf) + 4 * len(dat)


@pytest.mark.parametrize("row", _table2_rows(), ids=lambda r: "%d-%d" % (r[0], r[1]))
def test_table2_costs(row):
    lo, hi, bits = row
    probes = {lo, hi - 1, (lo + hi - 1) // 2}
    for v in probes:
        if v < 2 ** 32:
            assert _cost_bits(v) == bits, v


def test_info_nibble_values():
    # values 2..9 are carried in the info nibble as v + 6 (8..15), larger ones
    # carry their nibble count minus one (0..7): the two ranges never collide
    for v in range(2, 10):
        _, inf, dat = oracle.block_symbols([v])
        assert inf == [v + 6] and dat == []
    for v, nn in [(10, 1), (15, 1), (16, 2), (255, 2), (256, 3), (2 ** 32 - 1, 8)]:
        _, inf, dat = oracle.block_symbols([v])
        assert inf == [nn - 1] and len(dat) == nn
        assert int("".join("%X" % d for d in dat), 16) == v


def test_zero_difference_rejected():
    with pytest.raises(ValueError):
        oracle.block_symbols([1, 0, 3])


def _random_list(rng, n, universe):
    if n == 0:
        return np.zeros(0, np.uint32)
    return np.sort(rng.choice(universe, size=n, replace=False)).astype(np.uint32)


@pytest.mark.parametrize("cs", [4, 8, 16])
@pytest.mark.parametrize("compress", [True, False])
def test_roundtrip_fuzz(cs, compress):
    rng = np.random.default_rng(1234 + cs)
    nsub = 64 // cs
    for trial in range(60):
        n = int(rng.choice([0, 1, 2, 63, 64, 65, 127, 128, 129, 300, 1000]))
        universe = int(rng.choice([n + 1, 2 * n + 3, 10 ** 4, 10 ** 6, 2 ** 32 - 1]))
        universe = max(universe, n)
        j = _random_list(rng, n, universe)
        if trial % 7 == 0 and n > 2:  # force the extremes: first index 0 and 2^32-2
            j[0] = 0
            j[-1] = 2 ** 32 - 2
            j = np.unique(j)
            n = j.shape[0]
        m = rng.integers(1, 2 ** nsub, size=n).astype(np.uint16)
        w = oracle.encode_sc(j, m, cs, compress)
        jj, mm, used = oracle.decode_sc(w, n, cs, compress)
        assert used == w.shape[0]
        np.testing.assert_array_equal(jj, j)
        np.testing.assert_array_equal(mm, m)


def test_compressed_size_matches_table2():
    # total stream size = mask area + per segment (8-byte bitmask + Table II
    # nibble costs, padded to 4 bytes)
    rng = np.random.default_rng(7)
    for _ in range(30):
        n = int(rng.integers(1, 400))
        j = _random_list(rng, n, 5000)
        m = np.ones(n, np.uint16)
        w = oracle.encode_sc(j, m, 8, True)
        diffs = np.diff(np.concatenate([[-1], j.astype(np.int64)]))
        words = (n + 3) // 4
        for b in range(0, n, 64):
            blk = diffs[b:b + 64]
            nib_bits = sum(_cost_bits(int(v)) - 1 for v in blk)
            assert nib_bits % 4 == 0
            words += 2 + (nib_bits // 4 + 7) // 8
        assert w.shape[0] == words


def test_layout_bytes_by_hand():
    # j = [0, 1, 2, 12]: differences from -1 are 1, 1, 1, 10. Bitmask bit 3;
    # info nibble 0 (one data nibble), data nibble A; stream byte 0 = 0xA0.
    j = np.array([0, 1, 2, 12], np.uint32)
    m = np.array([0x01, 0x80, 0xFF, 0x10], np.uint16)
    w = oracle.encode_sc(j, m, 8, True)
    assert list(w) == [0x10FF8001, 0x00000008, 0x00000000, 0x000000A0]
