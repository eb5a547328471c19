"""sfc_sort_noalloc (the sort on the library's fixed device scratch) against
sfc_sort with a caller workspace: keys and order bit for bit, on two calls in a
row with the second smaller, plus the size limit."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    pts = rng.random((3, n), dtype=np.float64).astype(np.float32)
    # a few exact duplicates so that equal keys must keep input order
    if n > 16:
        pts[:, n // 2: n // 2 + 8] = pts[:, :8]
    dev = torch.device("cuda:0")
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in pts]


def _noalloc(ctx, x, y, z, box):
    n = x.numel()
    keys = ctx.empty(max(n, 1), torch.int64)
    perm = ctx.empty(max(n, 1), torch.int32)
    hb = (C.c_float * 6)(*box)
    rc = ctx.lib.sfc_sort_noalloc(ctx.handle, n, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                  C.c_void_p(z.data_ptr()), hb, C.c_void_p(keys.data_ptr()),
                                  C.c_void_p(perm.data_ptr()))
    return rc, keys[:n], perm[:n]


def test_noalloc_matches_workspace_sort_twice():
    _need_gpu()
    import paper_2602_19873_amd as sf
    torch.cuda.set_device(0)
    ctx = sf.Context(0)
    box = (0.0, 1.0, 0.0, 1.0, 0.0, 1.0)
    # the largest size, then a smaller ragged one: the second call must not
    # see anything of the first
    for n, seed in ((sf.SORT_NOALLOC_MAX_N, 11), (77_777, 12)):
        print("sfc_sort_noalloc n=%d seed=%d" % (n, seed), flush=True)
        x, y, z = _inputs(n, seed)
        k_ref, p_ref = sf.sfc_sort(ctx, x, y, z, box)
        rc, k, p = _noalloc(ctx, x, y, z, box)
        assert rc == 0, ctx.lib.sfcnl_last_error(ctx.handle).decode()
        torch.cuda.synchronize()
        assert torch.equal(k, k_ref)
        assert torch.equal(p, p_ref)
        # and the order really is the stable key order
        kh = k.cpu().numpy().view(np.uint64)
        ph = p.cpu().numpy()
        assert np.all(kh[1:] >= kh[:-1])
        tie = kh[1:] == kh[:-1]
        assert np.all(ph[1:][tie] > ph[:-1][tie])
        assert np.array_equal(np.sort(ph), np.arange(n, dtype=np.int32))
    ctx.close()


def test_noalloc_limits():
    _need_gpu()
    import paper_2602_19873_amd as sf
    from paper_2602_19873_amd import _lib
    torch.cuda.set_device(0)
    ctx = sf.Context(0)
    box = (0.0, 1.0, 0.0, 1.0, 0.0, 1.0)
    x, y, z = _inputs(16, 3)
    hb = (C.c_float * 6)(*box)
    big = sf.SORT_NOALLOC_MAX_N + 1
    rc = ctx.lib.sfc_sort_noalloc(ctx.handle, big, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                  C.c_void_p(z.data_ptr()), hb, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()))
    assert rc == _lib.E_ARG
    assert b"maximum" in ctx.lib.sfcnl_last_error(ctx.handle)
    rc, _, _ = _noalloc(ctx, x[:0], y[:0], z[:0], box)
    assert rc == 0
    # one particle
    rc, k, p = _noalloc(ctx, x[:1], y[:1], z[:1], box)
    assert rc == 0
    k_ref, p_ref = sf.sfc_sort(ctx, x[:1].contiguous(), y[:1].contiguous(), z[:1].contiguous(), box)
    torch.cuda.synchronize()
    assert torch.equal(k, k_ref) and int(p[0]) == 0
    ctx.close()
