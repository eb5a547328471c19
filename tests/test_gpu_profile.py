"""Stage timing (sfcnl_profile_begin / _end / _stages) on the whole path: every
stage of a step reports one bracketed call per step, a stage mask limits the
events to the named stages (the others report no calls) and the bench's
timed steps rely on that; mask bits past the stages are an argument error."""
import sys

import numpy as np
import pytest

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
    ctx.profile_stages(None)
    ctx.close()


def _pipe(sf, ctx, torch, n=50_000, half=True):
    s = workloads.uniform_varied(n, workloads.SEED_BASE + 41, target=60)
    x, y, z, h = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (s.x, s.y, s.z, s.h))
    pipe = sf.Pipeline(ctx, s.n, s.box, half=half)
    pipe.step(x, y, z, h)  # sizes the buffers (the synchronous build)
    torch.cuda.synchronize()
    return pipe, (x, y, z, h)


def test_every_stage_once_per_step(env):
    sf, ctx, torch = env
    pipe, f = _pipe(sf, ctx, torch)
    print("profile: all stages, 3 steps", flush=True)
    ctx.profile_stages(None)
    ctx.profile_begin(3)
    for _ in range(3):
        pipe.step(*f)
    prof = ctx.profile_end()
    for name, (ms, calls) in prof.items():
        assert calls == 3, (name, calls)
        assert ms > 0.0, name


@pytest.mark.parametrize("stages", [["traverse"], ["sort", "pass"], []])
def test_stage_mask(env, stages):
    sf, ctx, torch = env
    pipe, f = _pipe(sf, ctx, torch)
    print("profile: stages %s" % stages, flush=True)
    ctx.profile_stages(stages)
    try:
        ctx.profile_begin(2)
        for _ in range(2):
            pipe.step(*f)
        prof = ctx.profile_end()
    finally:
        ctx.profile_stages(None)
    for name, (ms, calls) in prof.items():
        if name in stages:
            assert calls == 2 and ms > 0.0, (name, calls, ms)
        else:
            assert calls == 0, (name, calls)


def test_stage_mask_arguments(env):
    sf, ctx, torch = env
    from paper_2602_19873_amd import _lib
    rc = ctx.lib.sfcnl_profile_stages(ctx.handle, 1 << _lib.NSTAGE)
    assert rc == _lib.E_ARG
    assert ctx.lib.sfcnl_profile_stages(None, 1) == _lib.E_ARG
    with pytest.raises(ValueError):
        ctx.profile_stages(["no such stage"])
    ctx.profile_stages(None)
