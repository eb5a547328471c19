"""Batched systems on the GPU: every system of a batch must get exactly what
the single-system calls give it on its own (keys, order, list words, density,
counts, iterated radii), with and without graph replay, and the iterated
counts must be the oracle's."""
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


def _systems(sizes, target, seed0):
    out = []
    for k, n in enumerate(sizes):
        if k % 2 == 0:
            s = workloads.uniform_varied(n, seed0 + k, target=target)
        else:
            s = workloads.plummer(n, seed0 + k, target=target)
        out.append(s)
    return out


# uneven sizes: an empty system, one below a super-cluster, ragged tails,
# several thousand particles (many octree levels)
SIZES = [3000, 0, 37, 20000, 64, 9001, 1, 15000]
# systems whose list words and densities are also checked against the oracle
# (one uniform, one Plummer)
ORACLE_SYS = (0, 5)
# for the iteration every system must hold more than target + 1 particles
SIZES_IT = [3000, 0, 300, 20000, 129, 9001, 15000]


def _concat(torch, systems, field):
    a = [getattr(s, field) for s in systems if s.n]
    return torch.from_numpy(np.ascontiguousarray(np.concatenate(a))).cuda()


def _batch(sf, ctx, systems):
    return sf.Batch(ctx, [s.n for s in systems], [s.box for s in systems])


def _single(sf, ctx, torch, s, h=None):
    from paper_2602_19873_amd import hseed
    return hseed.sorted_system(ctx, s, h)


def test_layout_and_sort_match_single(env):
    sf, ctx, torch = env
    systems = _systems(SIZES, 150, 500)
    b = _batch(sf, ctx, systems)
    assert b.n_in == sum(SIZES)
    assert np.all(b.pbase % 64 == 0)
    assert np.array_equal(np.diff(b.pbase), (np.array(SIZES) + 63) // 64 * 64)
    keys, perm = sf.batch_sort(ctx, b, *(_concat(torch, systems, f) for f in "xyz"))
    kh = keys.cpu().numpy().view(np.uint64)
    ph = perm.cpu().numpy().view(np.uint32)
    for s, sy in enumerate(systems):
        lo, n = int(b.pbase[s]), sy.n
        pad = slice(lo + n, int(b.pbase[s + 1]))
        assert np.all(kh[pad] == np.uint64(0xFFFFFFFFFFFFFFFF)) and np.all(ph[pad] == 0xFFFFFFFF)
        if n == 0:
            continue
        dev = torch.device("cuda:0")
        x, y, z = (torch.from_numpy(a).to(dev) for a in (sy.x, sy.y, sy.z))
        k1, p1 = sf.sfc_sort(ctx, x, y, z, sy.box)
        np.testing.assert_array_equal(kh[lo:lo + n], k1.cpu().numpy().view(np.uint64))
        np.testing.assert_array_equal(ph[lo:lo + n].astype(np.int64) - int(b.in_off[s]),
                                      p1.cpu().numpy().view(np.uint32).astype(np.int64))
        # and the oracle's keys and stable order
        ko = oracle.hilbert_keys(sy.x, sy.y, sy.z, sy.box)
        np.testing.assert_array_equal(kh[lo:lo + n], np.sort(ko, kind="stable"))


def _batch_arrays(sf, ctx, torch, b, systems):
    keys, perm = sf.batch_sort(ctx, b, *(_concat(torch, systems, f) for f in "xyz"))
    xs, ys, zs, hs = sf.batch_gather(ctx, b, perm, [_concat(torch, systems, f) for f in "xyzh"])
    return keys, xs, ys, zs, hs


@pytest.mark.parametrize("cs,half", [(8, False), (4, False), (16, False), (8, True), (4, True)])
def test_list_density_counts_match_single(env, cs, half):
    sf, ctx, torch = env
    systems = _systems(SIZES, 150, 600)
    b = _batch(sf, ctx, systems)
    keys, xs, ys, zs, hs = _batch_arrays(sf, ctx, torch, b, systems)
    hp = hs.cpu().numpy()
    for s, sy in enumerate(systems):
        lo, hi = int(b.pbase[s]), int(b.pbase[s + 1])
        assert np.all(np.isnan(hp[lo + sy.n:hi]))
    bbox = sf.batch_build_clusters(ctx, b, xs, ys, zs, hs, cluster_size=cs)
    nl = sf.batch_build_nlist(ctx, b, keys, xs, ys, zs, hs, bbox, pool=ctx.empty(1024, torch.int32),
                              cluster_size=cs, half=half)
    rho, nnb = sf.batch_pass(ctx, b, nl, xs, ys, zs, hs)
    info = nl.sc_info.cpu().numpy().view(np.uint32)
    pool = nl.pool.cpu().numpy().view(np.uint32)
    rho_h, nnb_h = rho.cpu().numpy(), nnb.cpu().numpy()
    total_words = 0
    for s, sy in enumerate(systems):
        if sy.n == 0:
            continue
        lo = int(b.pbase[s])
        c0, c1 = b.sc_range(s)
        k1, x1, y1, z1, h1 = _single(sf, ctx, torch, sy)
        bb1 = sf.build_clusters(ctx, x1, y1, z1, h1, cs)
        np.testing.assert_array_equal(bbox.cpu().numpy()[lo // cs: lo // cs + bb1.shape[0]], bb1.cpu().numpy())
        nl1 = sf.build_nlist(ctx, k1, x1, y1, z1, h1, bb1, cluster_size=cs, half=half)
        r1, n1 = sf.nlist_pass(ctx, nl1, x1, y1, z1, h1)
        i1 = nl1.sc_info.cpu().numpy().view(np.uint32)
        np.testing.assert_array_equal(info[c0:c1, 1], i1[:, 1])
        base = int(info[c0, 0])
        np.testing.assert_array_equal(info[c0:c1, 0] - base, i1[:, 0])
        words = nl1.used_bytes // 4
        np.testing.assert_array_equal(pool[base:base + words], nl1.pool.cpu().numpy().view(np.uint32)[:words])
        total_words += words
        if half:  # atomic summation order: equal within rounding
            np.testing.assert_allclose(rho_h[lo:lo + sy.n], r1.cpu().numpy(), rtol=2e-6, atol=0)
        else:
            np.testing.assert_array_equal(rho_h[lo:lo + sy.n], r1.cpu().numpy())
        np.testing.assert_array_equal(nnb_h[lo:lo + sy.n], n1.cpu().numpy())
        if sy.n <= 20000 and cs == 8:  # the oracle's counts for the same radii
            _, cnt = oracle.density(x1.cpu().numpy(), y1.cpu().numpy(), z1.cpu().numpy(), h1.cpu().numpy(), None,
                                    "grid")
            np.testing.assert_array_equal(n1.cpu().numpy(), cnt)
        if s in ORACLE_SYS:  # the batch's own words and densities against the oracle
            xa, ya, za, ha = (t.cpu().numpy() for t in (x1, y1, z1, h1))
            offs, jj, mm = oracle.cluster_list(xa, ya, za, ha, cs, "grid", half=half)
            oinfo, opool = oracle.encode_all(offs, jj, mm, cs, True)
            np.testing.assert_array_equal(info[c0:c1, 1], oinfo[:, 1])
            np.testing.assert_array_equal(info[c0:c1, 0] - base, oinfo[:, 0])
            np.testing.assert_array_equal(pool[base:base + words], opool)
            orho, ocnt = oracle.density(xa, ya, za, ha, None, "grid")
            np.testing.assert_array_equal(nnb_h[lo:lo + sy.n], ocnt)
            rel = np.abs(rho_h[lo:lo + sy.n].astype(np.float64) - orho) / orho
            assert rel.max() <= 1e-5, (s, rel.max())
    assert nl.used_bytes == 4 * total_words


@pytest.mark.parametrize("cs", [4, 8, 16])
def test_half_pass_masses(env, cs):
    """Non-unit masses through the batched symmetric pass: system sizes not
    divisible by the cluster size leave NaN padding in the last clusters,
    which must add nothing (rho of every real particle finite and equal to
    the single-system half pass and to the oracle)."""
    sf, ctx, torch = env
    sizes = [3001, 37, 9005, 1, 4099]
    systems = _systems(sizes, 150, 650)
    rng = np.random.default_rng(651)
    for sy in systems:
        sy.m = rng.uniform(0.5, 2.0, sy.n).astype(np.float32)
    b = _batch(sf, ctx, systems)
    keys, perm = sf.batch_sort(ctx, b, *(_concat(torch, systems, f) for f in "xyz"))
    xs, ys, zs, hs, ms = sf.batch_gather(ctx, b, perm, [_concat(torch, systems, f) for f in "xyzhm"])
    assert np.all(np.isnan(ms.cpu().numpy()[int(b.pbase[0]) + sizes[0]:int(b.pbase[1])]))
    bbox = sf.batch_build_clusters(ctx, b, xs, ys, zs, hs, cluster_size=cs)
    nl = sf.batch_build_nlist(ctx, b, keys, xs, ys, zs, hs, bbox, pool=ctx.empty(1024, torch.int32),
                              cluster_size=cs, half=True)
    rho, nnb = sf.batch_pass(ctx, b, nl, xs, ys, zs, hs, m=ms)
    rho_h, nnb_h = rho.cpu().numpy(), nnb.cpu().numpy()
    for s, sy in enumerate(systems):
        lo = int(b.pbase[s])
        got = rho_h[lo:lo + sy.n]
        assert np.all(np.isfinite(got)), s
        k1, p1 = sf.sfc_sort(ctx, *(torch.from_numpy(a).cuda() for a in (sy.x, sy.y, sy.z)), sy.box)
        x1, y1, z1, h1, m1 = sf.sfc_gather(ctx, p1, [torch.from_numpy(a).cuda() for a in (sy.x, sy.y, sy.z, sy.h,
                                                                                          sy.m)])
        bb1 = sf.build_clusters(ctx, x1, y1, z1, h1, cs)
        nl1 = sf.build_nlist(ctx, k1, x1, y1, z1, h1, bb1, cluster_size=cs, half=True)
        r1, n1 = sf.nlist_pass(ctx, nl1, x1, y1, z1, h1, m=m1)
        np.testing.assert_allclose(got, r1.cpu().numpy(), rtol=2e-6, atol=0)
        np.testing.assert_array_equal(nnb_h[lo:lo + sy.n], n1.cpu().numpy())
        orho, ocnt = oracle.density(*(t.cpu().numpy() for t in (x1, y1, z1, h1, m1)), "grid")
        np.testing.assert_array_equal(nnb_h[lo:lo + sy.n], ocnt)
        rel = np.abs(got.astype(np.float64) - orho) / orho
        assert rel.max() <= 1e-5, (s, rel.max())


def _perturbed(systems, seed, spread=2.0):
    rng = np.random.default_rng(seed)
    for s in systems:
        if s.n:
            f = np.exp(rng.uniform(-np.log(spread), np.log(spread), s.n))
            s.h = (s.h * f).astype(np.float32)
    return systems


@pytest.mark.parametrize("use_graph,recount", [(True, 0), (False, 0), (True, 1), (True, 2)])
def test_h_iterate_matches_single(env, use_graph, recount):
    sf, ctx, torch = env
    T = 60
    systems = _perturbed(_systems(SIZES_IT, T, 700), 701)
    b = _batch(sf, ctx, systems)
    keys, xs, ys, zs, hs = _batch_arrays(sf, ctx, torch, b, systems)
    res = sf.batch_h_iterate(ctx, b, keys, xs, ys, zs, hs, target=T, tol=1, use_graph=use_graph, recount=recount)
    _say("batch: %d rounds, per system %s" % (res.iters, res.sys_rounds.tolist()))
    assert res.converged and res.unconverged == 0
    hb, nb = hs.cpu().numpy(), res.nnb.cpu().numpy()
    for s, sy in enumerate(systems):
        if sy.n == 0:
            assert res.sys_rounds[s] == 1
            continue
        lo = int(b.pbase[s])
        k1, x1, y1, z1, h1 = _single(sf, ctx, torch, sy)
        r1 = sf.h_iterate(ctx, k1, x1, y1, z1, h1, target=T, tol=1)
        assert r1.converged
        np.testing.assert_array_equal(hb[lo:lo + sy.n], h1.cpu().numpy())
        np.testing.assert_array_equal(nb[lo:lo + sy.n], r1.nnb.cpu().numpy()[:sy.n])
        assert res.sys_rounds[s] == r1.iters, (s, res.sys_rounds[s], r1.iters)
    assert res.iters == max(int(r) for r in res.sys_rounds)
    # the converged counts are the oracle's, within the tolerance
    for s in (0, 3):
        sy = systems[s]
        lo = int(b.pbase[s])
        sl = slice(lo, lo + sy.n)
        _, cnt = oracle.density(xs.cpu().numpy()[sl], ys.cpu().numpy()[sl], zs.cpu().numpy()[sl], hb[sl], None,
                                "grid")
        np.testing.assert_array_equal(nb[sl], cnt)
        assert np.all(np.abs(cnt - T) <= 1)


def test_h_iterate_capacity_resume(env):
    """A pool too small for the list fails a round without touching h; the
    binding grows it and resumes, ending where an unconstrained run ends."""
    sf, ctx, torch = env
    T = 60
    systems = _perturbed(_systems([5000, 700, 12000], T, 800), 801)
    b = _batch(sf, ctx, systems)
    arrs = _batch_arrays(sf, ctx, torch, b, systems)
    h0 = arrs[4].clone()
    ref = sf.batch_h_iterate(ctx, b, *arrs, target=T)
    h_ref = arrs[4].cpu().numpy()
    arrs[4].copy_(h0)
    small = {"bracket": ctx.empty(2 * b.n_pad, torch.float32), "bbox": ctx.empty((b.n_pad // 8, 8), torch.float32),
             "sc_info": ctx.empty((b.n_pad // 64, 2), torch.int32), "pool": ctx.empty(256, torch.int32),
             "rho": ctx.empty(b.n_pad, torch.float32), "nnb": ctx.empty(b.n_pad, torch.int32), "max_j": 16}
    got = sf.batch_h_iterate(ctx, b, *arrs, target=T, bufs=small)
    assert small["pool"].numel() > 256 and small["max_j"] > 16
    assert got.converged and got.iters == ref.iters
    np.testing.assert_array_equal(arrs[4].cpu().numpy(), h_ref)


@pytest.mark.parametrize("mode", ["after_first", "before_first"])
def test_seeded_batch_matches_single(env, mode):
    """The learned step gives each system of a batch what it gives the
    system alone (per-system box edges, key searches inside the system)."""
    sf, ctx, torch = env
    sm = sf.SEED_AFTER_FIRST if mode == "after_first" else sf.SEED_BEFORE_FIRST
    from paper_2602_19873_amd import hseed
    T = 60
    systems = _perturbed(_systems([4000, 0, 9000, 130], T, 900), 901, spread=3.0)
    params = sf.mlp_init(ctx, 3)
    params.mul_(0.1)  # a small correction to the cube-root step
    b = _batch(sf, ctx, systems)
    keys, xs, ys, zs, hs = _batch_arrays(sf, ctx, torch, b, systems)
    res = sf.batch_h_iterate(ctx, b, keys, xs, ys, zs, hs, target=T, mlp_params=params, seed_mode=sm)
    assert res.converged
    hb = hs.cpu().numpy()
    for s, sy in enumerate(systems):
        if sy.n == 0:
            continue
        lo = int(b.pbase[s])
        k1, x1, y1, z1, h1 = _single(sf, ctx, torch, sy)
        r1 = sf.h_iterate(ctx, k1, x1, y1, z1, h1, target=T, tol=1, mlp_params=params,
                          box_edge=hseed.box_edge(sy.box), seed_mode=sm)
        assert r1.converged
        np.testing.assert_array_equal(hb[lo:lo + sy.n], h1.cpu().numpy())
        assert res.sys_rounds[s] == r1.iters


@pytest.mark.parametrize("max_iters", [3, 6, 7])
def test_round_limit_with_graph_replays(env, max_iters):
    """Rounds are replayed several per graph launch; a round limit that cuts
    through a replay still runs exactly max_iters rounds: the graph run ends
    with the radii, counts and unconverged total of the run without graphs."""
    sf, ctx, torch = env
    T = 60
    systems = _perturbed(_systems([6000, 300, 9000], T, 950), 951, spread=4.0)
    b = _batch(sf, ctx, systems)
    keys, xs, ys, zs, hs = _batch_arrays(sf, ctx, torch, b, systems)
    h0 = hs.clone()
    out = {}
    for use_graph in (True, False):
        hs.copy_(h0)
        res = sf.batch_h_iterate(ctx, b, keys, xs, ys, zs, hs, target=T, tol=1, max_iters=max_iters,
                                 use_graph=use_graph)
        out[use_graph] = (hs.cpu().numpy(), res.nnb.cpu().numpy(), res.unconverged, res.iters, res.converged)
    a, c = out[True], out[False]
    assert a[2:] == c[2:]
    np.testing.assert_array_equal(a[0], c[0])
    np.testing.assert_array_equal(a[1], c[1])
    assert a[3] <= max_iters and (a[4] or a[3] == max_iters)
