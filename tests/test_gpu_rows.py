"""Compressed 1x1 list on the GPU (build_rows, rows_pass) against the oracle,
through the C ABI: row headers and every pool word bit-exact, counts exact,
densities within 1e-5 relative. The oracle sees the generator's arrays in its
own SFC order; the GPU's permutation is checked equal to it first."""
import sys

import numpy as np
import pytest

import oracle
from paper_2602_19873_amd import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2602_19873_amd as sf
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    torch.cuda.set_device(0)
    ctx = sf.Context(0)
    yield sf, ctx, torch
    ctx.close()


def _system(n, seed, target, spread=0.4):
    rng = np.random.default_rng(seed)
    p = rng.random((3, n))
    h = workloads.radius_for_neighbours(n, target) * rng.uniform(1 - spread, 1 + spread, n)
    f = lambda a: np.ascontiguousarray(a.astype(np.float32))
    return workloads.ParticleSystem("rows_uniform", f(p[0]), f(p[1]), f(p[2]), f(h), None, workloads.UNIT_BOX)


def _run(env, s, cs, comp_in, comp, per=None, pool=None):
    sf, ctx, torch = env
    _say("rows case n=%d cs=%d list_compress=%d rows_compress=%d period=%s" % (s.n, cs, comp_in, comp, per))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    x, y, z, h = (dev(a) for a in (s.x, s.y, s.z, s.h))
    pipe = sf.Pipeline(ctx, s.n, s.box, comp_in, 64, 512, cluster_size=cs, half=False, period=per)
    nl = pipe.step(x, y, z, h, density=False)
    xs, ys, zs, hs = pipe.sorted[:4]
    rl = sf.build_rows(ctx, nl, xs, ys, zs, hs, compress=comp, pool=pool)
    rho, nnb = sf.rows_pass(ctx, rl, xs, ys, zs, hs)
    torch.cuda.synchronize()
    o = oracle.sfc_order(oracle.hilbert_keys(s.x, s.y, s.z, s.box))
    np.testing.assert_array_equal(pipe.perm.cpu().numpy().view(np.uint32), o)
    return rl, rho.cpu().numpy(), nnb.cpu().numpy(), (s.x[o], s.y[o], s.z[o], s.h[o])


def _compare(rl, rho, nnb, sorted_arrays, comp, per=None):
    xo, yo, zo, ho = sorted_arrays
    info, pool = oracle.row_list(xo, yo, zo, ho, comp, period=per)
    np.testing.assert_array_equal(rl.row_info.cpu().numpy().view(np.uint32), info)
    assert rl.used_bytes == 4 * pool.shape[0]
    np.testing.assert_array_equal(rl.pool.cpu().numpy().view(np.uint32)[: pool.shape[0]], pool)
    r, c = oracle.density(xo, yo, zo, ho, period=per)
    np.testing.assert_array_equal(nnb, c)
    rel = np.abs(rho.astype(np.float64) - r) / r
    assert rel.max() <= 1e-5, "density error %.3g" % rel.max()


@pytest.mark.parametrize("cs,comp_in,comp", [(8, True, True), (8, False, True), (8, True, False), (4, True, True),
                                             (16, True, True), (16, False, False)])
def test_rows_match_oracle(env, cs, comp_in, comp):
    s = _system(20011, 601, 60)
    rl, rho, nnb, so = _run(env, s, cs, comp_in, comp)
    _compare(rl, rho, nnb, so, comp)


@pytest.mark.parametrize("n", [1, 65, 200, 4099])
def test_rows_small_and_ragged(env, n):
    s = _system(n, 602 + n, 40)
    rl, rho, nnb, so = _run(env, s, 8, True, True)
    _compare(rl, rho, nnb, so, True)


def test_rows_periodic(env):
    per = (1.0, 1.0, 1.0)
    s = _system(20011, 603, 60)
    rl, rho, nnb, so = _run(env, s, 8, True, True, per=per)
    _compare(rl, rho, nnb, so, True, per=per)


def test_rows_capacity_retry(env):
    sf, ctx, torch = env
    s = _system(5000, 604, 60)
    small = torch.empty(64, dtype=torch.int32, device="cuda")
    rl, rho, nnb, so = _run(env, s, 8, True, True, pool=small)
    assert rl.pool.numel() > 64
    _compare(rl, rho, nnb, so, True)
    # without growing, the call reports the size needed
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    x, y, z, h = (dev(a) for a in (s.x, s.y, s.z, s.h))
    pipe = sf.Pipeline(ctx, s.n, s.box, True, 64, 512, cluster_size=8, half=False)
    nl = pipe.step(x, y, z, h, density=False)
    with pytest.raises(sf.SfcnlError) as e:
        sf.build_rows(ctx, nl, *pipe.sorted[:4], pool=small, grow=False)
    assert e.value.code == -3


def test_rows_100k(env):
    s = _system(100000, 605, 100, spread=0.2)
    rl, rho, nnb, so = _run(env, s, 8, True, True)
    _compare(rl, rho, nnb, so, True)
    _say("100k rows: %.2f B/particle" % rl.bytes_per_particle())
