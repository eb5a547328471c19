"""build_nlist_async / build_nlist_result against the waiting build_nlist and
the oracle: the same list bytes and sizes, a pass enqueued before the result
reads a complete list, capacity errors leave every list inside the pool."""
import sys

import numpy as np
import pytest

import oracle
from paper_2602_19873_amd import workloads

pytestmark = pytest.mark.gpu


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


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("half", [False, True])
@pytest.mark.parametrize("n", [5000, 33333])
def test_pipeline_steps_after_the_first_match_oracle(env, half, n):
    sf, ctx, torch = env
    _say("case n=%d half=%d" % (n, half))
    s = workloads.uniform_varied(n, 4100 + n, target=60.0)
    x, y, z, h = (_dev(torch, a) for a in (s.x, s.y, s.z, s.h))
    pipe = sf.Pipeline(ctx, s.n, s.box, half=half)
    first = pipe.step(x, y, z, h)
    torch.cuda.synchronize()
    pool1 = _u32(first.pool)[: first.used_bytes // 4].copy()
    for _ in range(2):  # later steps take the asynchronous build
        nl = pipe.step(x, y, z, h)
        torch.cuda.synchronize()
        assert not nl.pending and nl.used_bytes == first.used_bytes and nl.max_nj == first.max_nj
        np.testing.assert_array_equal(_u32(nl.pool)[: nl.used_bytes // 4], pool1)
    ref = oracle.pipeline(s.x, s.y, s.z, s.h, s.box, None, 8, True, "grid", half=half)
    np.testing.assert_array_equal(pool1, ref["pool"])
    np.testing.assert_array_equal(pipe.nnb.cpu().numpy()[: s.n], ref["nnb"])
    rel = np.abs(pipe.rho.cpu().numpy()[: s.n].astype(np.float64) - ref["rho"]) / ref["rho"]
    assert rel.max() <= 1e-5, rel.max()


def test_async_capacity_error_keeps_the_pass_inside_the_pool(env):
    sf, ctx, torch = env
    s = workloads.uniform_varied(20000, 4201, target=80.0)
    x, y, z, h = (_dev(torch, a) for a in (s.x, s.y, s.z, s.h))
    keys, perm = sf.sfc_sort(ctx, x, y, z, s.box)
    xs, ys, zs, hs = sf.sfc_gather(ctx, perm, [x, y, z, h])
    bbox = sf.build_clusters(ctx, xs, ys, zs, hs)
    full = sf.build_nlist(ctx, keys, xs, ys, zs, hs, bbox)
    torch.cuda.synchronize()
    nsc = (s.n + 63) // 64
    small = torch.zeros(full.used_bytes // 8, dtype=torch.int32, device="cuda")  # half the words needed
    sc_info = torch.empty((nsc, 2), dtype=torch.int32, device="cuda")
    _say("case capacity: pool %d of %d bytes" % (small.numel() * 4, full.used_bytes))
    nl = sf.build_nlist_async(ctx, keys, xs, ys, zs, hs, bbox, small, full.ws, sc_info)
    rho, nnb = sf.nlist_pass(ctx, nl, xs, ys, zs, hs)  # enqueued before the result: must stay in the pool
    assert sf.build_nlist_finish(ctx, nl) is False
    assert nl.used_bytes == full.used_bytes and nl.max_nj == full.max_nj
    torch.cuda.synchronize()
    info = _u32(sc_info).reshape(-1, 2)
    off, cnt = info[:, 0].astype(np.int64), info[:, 1]
    assert (cnt == 0).any() and (cnt > 0).any()
    fit = cnt > 0
    assert (off[fit] < small.numel()).all()
    # a retry with room gives the waiting build's list
    big = torch.zeros(full.used_bytes // 4 + 16, dtype=torch.int32, device="cuda")
    nl2 = sf.build_nlist_async(ctx, keys, xs, ys, zs, hs, bbox, big, full.ws, sc_info)
    assert sf.build_nlist_finish(ctx, nl2) is True
    np.testing.assert_array_equal(_u32(big)[: nl2.used_bytes // 4], _u32(full.pool)[: full.used_bytes // 4])


def test_result_without_pending_build_is_an_argument_error(env):
    sf, ctx, torch = env
    import ctypes as C
    used, maxnj = C.c_size_t(), C.c_int64()
    assert ctx.lib.build_nlist_result(ctx.handle, C.byref(used), C.byref(maxnj)) == -1


def test_async_build_of_nothing(env):
    sf, ctx, torch = env
    import ctypes as C
    from paper_2602_19873_amd import _lib
    o = sf._opts(8, True, 128, 512, False, None)
    assert ctx.lib.build_nlist_async(ctx.handle, 0, None, None, None, None, None, None, C.byref(o), None, 0,
                                     None, None, 0) == 0
    used, maxnj = C.c_size_t(7), C.c_int64(7)
    assert ctx.lib.build_nlist_result(ctx.handle, C.byref(used), C.byref(maxnj)) == 0
    assert used.value == 0 and maxnj.value == 0
    assert ctx.lib.build_nlist_result(ctx.handle, C.byref(used), C.byref(maxnj)) == _lib.E_ARG
