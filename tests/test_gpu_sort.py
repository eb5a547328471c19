"""SFC sort (Sec. II-A: Hilbert order) on inputs that drive its long-run paths:
particles packed into cells of the top 24 key bits (octree level 8), so that
runs of equal prefixes are longer than a count-placed run (sorted by LDS radix
passes) or than the LDS capacity (sorted by one block through global memory,
with an even or an odd number of passes), such clusters inside a uniform
background, and all particles at one point. Keys and order must equal the
oracle's keys and a stable argsort of them, bit for bit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402

pytestmark = pytest.mark.gpu

BOX = (0.0, 1.0, 0.0, 1.0, 0.0, 1.0)


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2602_19873_amd as sf
    torch.cuda.set_device(0)
    ctx = sf.Context(0)
    yield sf, ctx
    ctx.close()


def _cluster(rng, n, corner, side):
    """n points uniform in the cube [corner, corner + side)^3 (float64, then f32)."""
    return (np.asarray(corner)[:, None] + side * rng.random((3, n))).astype(np.float32)


def _check(sf, ctx, pts):
    dev = torch.device("cuda:0")
    x, y, z = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in pts)
    print("sort n=%d" % pts.shape[1], flush=True)
    keys, perm = sf.sfc_sort(ctx, x, y, z, BOX)
    torch.cuda.synchronize()
    ko = oracle.hilbert_keys(pts[0], pts[1], pts[2], BOX)
    po = np.argsort(ko, kind="stable").astype(np.uint32)
    assert np.array_equal(perm.cpu().numpy().view(np.uint32), po)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), ko[po])


def test_long_runs_odd_passes(env):
    # one level-7 cell filled: eight runs of ~7,500 (its level-8 cells), keys
    # differing in bits 0..38 (five passes, the result copied back from the
    # temporary range)
    sf, ctx = env
    rng = np.random.default_rng(7001)
    _check(sf, ctx, _cluster(rng, 60_000, (0.3125, 0.5, 0.1875), 2.0 ** -7))


def test_one_long_run_even_passes(env):
    # one level-11 cell filled: one run, keys differing in bits 0..29 (four
    # passes)
    sf, ctx = env
    rng = np.random.default_rng(7002)
    _check(sf, ctx, _cluster(rng, 9_000, (0.625, 0.25, 0.75), 2.0 ** -11))


def test_long_runs_in_uniform_background(env):
    sf, ctx = env
    rng = np.random.default_rng(7003)
    pts = np.concatenate([rng.random((3, 70_000)).astype(np.float32),
                          _cluster(rng, 20_000, (0.5, 0.5, 0.5), 2.0 ** -8),
                          _cluster(rng, 5_000, (0.125, 0.875, 0.25), 2.0 ** -9),
                          _cluster(rng, 4_100, (0.0625, 0.0625, 0.9375), 2.0 ** -10),
                          _cluster(rng, 1_500, (0.75, 0.125, 0.5), 2.0 ** -9),
                          _cluster(rng, 100, (0.875, 0.625, 0.0625), 2.0 ** -12),
                          _cluster(rng, 65, (0.25, 0.375, 0.625), 2.0 ** -12)], axis=1)
    pts = pts[:, rng.permutation(pts.shape[1])]
    _check(sf, ctx, np.ascontiguousarray(pts))


def test_all_at_one_point(env):
    sf, ctx = env
    pts = np.full((3, 12_345), 0.4, dtype=np.float32)
    _check(sf, ctx, pts)


@pytest.mark.parametrize("n", [1, 2, 63, 2047, 2048, 2049, 4097, 100_003])
def test_sizes_across_tiles(env, n):
    sf, ctx = env
    rng = np.random.default_rng(7100 + n)
    _check(sf, ctx, rng.random((3, n)).astype(np.float32))
