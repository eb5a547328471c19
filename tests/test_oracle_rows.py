"""Pins of the oracle's compressed 1x1 list (the combination of the index
compression with a full neighbour list that the paper names as future work,
Sec. V).

A row is the index stream of a super-cluster list without masks, so it must
equal the tail of the (separately pinned) super-cluster encoding of the same
indices; rows must decode to the pair set's rows, with and without periodic
boundaries."""
import numpy as np
import pytest

import oracle


def test_row_is_super_cluster_stream_without_masks():
    rng = np.random.default_rng(11)
    for n in (1, 5, 63, 64, 65, 200, 777):
        j = np.sort(rng.choice(2 ** 20, n, replace=False)).astype(np.uint32)
        j[: n // 2] = np.arange(n // 2, dtype=np.uint32) + j[0]  # a run of ones
        j = np.unique(j)
        for cs, mwords in ((8, (len(j) + 3) // 4), (4, (2 * len(j) + 3) // 4)):
            m = rng.integers(0, 256 if cs == 8 else 65536, len(j)).astype(np.uint16)
            sc = oracle.encode_sc(j, m, cs, True)
            np.testing.assert_array_equal(oracle.encode_row(j, True), sc[mwords:])
        np.testing.assert_array_equal(oracle.encode_row(j, False), j)
        for comp in (True, False):
            back, used = oracle.decode_row(oracle.encode_row(j, comp), len(j), comp)
            np.testing.assert_array_equal(back, j)


def test_consecutive_row_is_two_words():
    # differences are taken from -1, so a row 0, 1, ..., 63 is all ones: an
    # empty nibble stream and a zero bit mask
    np.testing.assert_array_equal(oracle.encode_row(np.arange(64, dtype=np.uint32)), [0, 0])
    # starting at 5: one info nibble (6 -> 12) in the first word after the mask
    np.testing.assert_array_equal(oracle.encode_row(np.arange(5, 69, dtype=np.uint32)), [1, 0, 12])


@pytest.mark.parametrize("period", [None, (1.0, 1.0, 0.0)])
def test_row_list_decodes_to_pair_rows(period):
    rng = np.random.default_rng(12)
    n = 3000
    x, y, z = (rng.random(n).astype(np.float32) for _ in range(3))
    h = (0.05 * rng.uniform(0.5, 1.5, n)).astype(np.float32)
    h[7] = np.float32(1e-6)  # an isolated particle keeps an empty row unless a large radius reaches it
    offs, nbr = oracle.pairs_csr(x, y, z, h, "grid", period=period)
    for comp in (True, False):
        info, pool = oracle.row_list(x, y, z, h, comp, period=period)
        assert info[0, 0] == 0
        for i in range(n):
            o, c = int(info[i, 0]), int(info[i, 1])
            assert c == offs[i + 1] - offs[i]
            end = int(info[i + 1, 0]) if i + 1 < n else pool.shape[0]
            row, used = oracle.decode_row(pool[o:end], c, comp)
            assert used == end - o
            np.testing.assert_array_equal(row, nbr[offs[i]:offs[i + 1]])
