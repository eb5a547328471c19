"""The two gather forms (direct, and staged through 16-byte records) against
the definition out[f][k] = in[f][perm[k]], bit for bit."""
import sys

import numpy as np
import pytest

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


@pytest.mark.parametrize("n", [1, 255, 256, 70001])
@pytest.mark.parametrize("nf", [1, 2, 3, 4, 5, 8])
def test_staged_gather_matches_definition(env, n, nf):
    sf, ctx, torch = env
    print("case n=%d nf=%d" % (n, nf), flush=True)
    sys.stdout.flush()
    rng = np.random.default_rng(1000 + 7 * n + nf)
    perm = rng.permutation(n).astype(np.uint32)
    fields = [rng.standard_normal(n).astype(np.float32) for _ in range(nf)]
    fields[0][: min(n, 3)] = [np.nan, -0.0, np.inf][: min(n, 3)]  # bit patterns travel unchanged
    dp = torch.from_numpy(perm.view(np.int32)).cuda()
    df = [torch.from_numpy(f).cuda() for f in fields]
    direct = sf.sfc_gather(ctx, dp, df)
    ws = torch.empty(sf.sfc_gather_workspace(n) + 3, dtype=torch.uint8, device="cuda")[3:]  # unaligned start
    staged = sf.sfc_gather(ctx, dp, df, ws=ws)
    torch.cuda.synchronize()
    for f, a, b in zip(fields, direct, staged):
        want = f[perm].view(np.uint32)
        np.testing.assert_array_equal(a.cpu().numpy().view(np.uint32), want)
        np.testing.assert_array_equal(b.cpu().numpy().view(np.uint32), want)


def test_staged_gather_reports_bad_perm_and_small_workspace(env):
    sf, ctx, torch = env
    n = 1000
    perm = np.arange(n, dtype=np.uint32)
    perm[10] = n + 5  # not a permutation: reported, never read outside
    dp = torch.from_numpy(perm.view(np.int32)).cuda()
    x = torch.arange(n, dtype=torch.float32, device="cuda")
    ws = torch.empty(sf.sfc_gather_workspace(n), dtype=torch.uint8, device="cuda")
    with pytest.raises(sf.SfcnlError) as ei:
        sf.sfc_gather(ctx, dp, [x, x.clone()], ws=ws)
        ctx.sync()
    assert ei.value.code == -2
    ctx.sync()  # latch cleared
    with pytest.raises(sf.SfcnlError) as ei:
        sf.sfc_gather(ctx, torch.arange(n, dtype=torch.int32, device="cuda"), [x, x.clone()], ws=ws[:100])
    assert ei.value.code == -1


def test_staged_gather_of_nothing(env):
    sf, ctx, torch = env
    import ctypes as C
    ins = (C.c_void_p * 1)(None)
    outs = (C.c_void_p * 1)(None)
    assert ctx.lib.sfc_gather_ws(ctx.handle, 0, None, 1, ins, outs, None, 0) == 0
