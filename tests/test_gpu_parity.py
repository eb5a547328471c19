"""GPU path against the CPU oracle, through the C ABI.

Bar: keys, order, boxes, list headers and list bytes bit-exact; neighbour
counts exact; FP32 densities within 1e-5 relative of the FP64 oracle.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2602_19873_amd import workloads

pytestmark = pytest.mark.gpu

RHO_RTOL = 1e-5


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


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _run(env, s, compress=True, leaf_bucket=64, max_j=512, mass=None, cs=8, half=False):
    sf, ctx, torch = env
    _say("case %s n=%d compress=%d bucket=%d cs=%d half=%d" % (s.name, s.n, compress, leaf_bucket, cs, half))
    x, y, z, h = (_dev(torch, a) for a in (s.x, s.y, s.z, s.h))
    m = None if mass is None else _dev(torch, mass)
    pipe = sf.Pipeline(ctx, s.n, s.box, compress, leaf_bucket, max_j, with_mass=mass is not None, cluster_size=cs,
                       half=half)
    nl = pipe.step(x, y, z, h, m)
    torch.cuda.synchronize()
    out = dict(keys=pipe.keys.cpu().numpy().view(np.uint64), perm=_u32(pipe.perm),
               x=pipe.sorted[0].cpu().numpy(), h=pipe.sorted[3].cpu().numpy(),
               bbox=pipe.bbox.cpu().numpy(), sc_info=_u32(nl.sc_info).reshape(-1, 2),
               pool=_u32(nl.pool)[: nl.used_bytes // 4], rho=pipe.rho.cpu().numpy()[: s.n],
               nnb=pipe.nnb.cpu().numpy()[: s.n], nl=nl)
    return out


def _compare(s, g, compress=True, mass=None, method="grid", cs=8, half=False):
    ref = oracle.pipeline(s.x, s.y, s.z, s.h, s.box, mass, cs, compress, method, half=half)
    np.testing.assert_array_equal(g["keys"], ref["sorted_keys"])
    np.testing.assert_array_equal(g["perm"], ref["perm"])
    np.testing.assert_array_equal(g["x"], ref["x"])
    np.testing.assert_array_equal(g["h"], ref["h"])
    np.testing.assert_array_equal(g["bbox"], oracle.cluster_bboxes(ref["x"], ref["y"], ref["z"], ref["h"], cs))
    np.testing.assert_array_equal(g["sc_info"], ref["sc_info"])
    np.testing.assert_array_equal(g["pool"], ref["pool"])
    np.testing.assert_array_equal(g["nnb"], ref["nnb"])
    rel = np.abs(g["rho"].astype(np.float64) - ref["rho"]) / ref["rho"]
    assert rel.max() <= RHO_RTOL, rel.max()
    return ref


@pytest.mark.parametrize("compress", [True, False])
def test_uniform_32k(env, compress):
    s = workloads.make_config("uniform_32k")
    g = _run(env, s, compress)
    _compare(s, g, compress)


@pytest.mark.parametrize("n", [1, 7, 8, 9, 63, 64, 65, 200, 1000, 4099])
def test_small_and_ragged(env, n):
    s = workloads.uniform_varied(n, 1000 + n, target=40.0)
    _compare(s, _run(env, s))


@pytest.mark.parametrize("bucket", [8, 16, 32, 128, 256])
def test_leaf_bucket_does_not_change_list(env, bucket):
    s = workloads.uniform_varied(20000, 31, target=80.0)
    _compare(s, _run(env, s, leaf_bucket=bucket))


def test_varied_radii_wide_spread(env):
    rng = np.random.default_rng(5)
    s = workloads.uniform_varied(30000, 6, target=60.0)
    s.h = (s.h * np.exp(rng.uniform(-1.2, 1.2, s.n))).astype(np.float32)
    _compare(s, _run(env, s))


def test_masses(env):
    s = workloads.uniform_varied(12000, 8, target=100.0)
    m = np.random.default_rng(3).uniform(0.1, 3.0, s.n).astype(np.float32)
    _compare(s, _run(env, s, mass=m), mass=m)


def test_evrard_sphere_small(env):
    s = workloads.evrard_sphere(60000, 17, target=100.0, seed_h="analytic")
    _compare(s, _run(env, s))


def test_plummer_small(env):
    s = workloads.plummer(40000, 19, target=150.0)
    _compare(s, _run(env, s))


def test_coincident_and_tied_keys(env):
    # many particles share a position (identical keys, d2 = 0) plus a few apart
    rng = np.random.default_rng(9)
    n = 3000
    base = rng.random((3, 40)).astype(np.float32)
    pick = rng.integers(0, 40, n)
    s = workloads.ParticleSystem("ties", base[0][pick].copy(), base[1][pick].copy(), base[2][pick].copy(),
                                 np.full(n, 0.05, np.float32), None, workloads.UNIT_BOX)
    _compare(s, _run(env, s))


def test_lattice_exact_radius(env):
    # d == R exactly on a lattice: the strict test rejects those pairs
    a = 0.125
    g = np.arange(8, dtype=np.float32) * np.float32(a)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    for hv in (0.125, 0.13, 0.18):
        s = workloads.ParticleSystem("lattice", X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy(),
                                     np.full(X.size, hv, np.float32), None, workloads.UNIT_BOX)
        _compare(s, _run(env, s), method="brute")


def test_huge_and_tiny_radius(env):
    rng = np.random.default_rng(4)
    n = 700
    x, y, z = (rng.random(n).astype(np.float32) for _ in range(3))
    for hv in (5.0, 1e-6):
        s = workloads.ParticleSystem("extreme", x, y, z, np.full(n, hv, np.float32), None, workloads.UNIT_BOX)
        _compare(s, _run(env, s), method="brute")


def test_device_decoder_matches_oracle_list(env):
    sf, ctx, torch = env
    s = workloads.uniform_varied(20000, 44, target=120.0)
    for compress in (True, False):
        g = _run(env, s, compress)
        offs, j, m = sf.nlist_decode(ctx, g["nl"])
        ref = oracle.pipeline(s.x, s.y, s.z, s.h, s.box, None, 8, compress)
        np.testing.assert_array_equal(offs, ref["offs"])
        np.testing.assert_array_equal(j, ref["j"])
        np.testing.assert_array_equal(m, ref["mask"])


# Cluster sizes 4 and 16 (64 / cs i-clusters per super-cluster, masks of 16
# and 4 bits): the same oracle comparisons as for size 8.
CS_OTHER = [4, 16]


@pytest.mark.parametrize("cs", CS_OTHER)
@pytest.mark.parametrize("compress", [True, False])
def test_cluster_size_uniform_32k(env, cs, compress):
    s = workloads.make_config("uniform_32k")
    _compare(s, _run(env, s, compress, cs=cs), compress, cs=cs)


@pytest.mark.parametrize("cs", CS_OTHER)
@pytest.mark.parametrize("n", [1, 5, 17, 63, 65, 1000, 4099])
def test_cluster_size_small_and_ragged(env, cs, n):
    s = workloads.uniform_varied(n, 2000 + n, target=40.0)
    _compare(s, _run(env, s, cs=cs), cs=cs)


@pytest.mark.parametrize("cs", CS_OTHER)
def test_cluster_size_varied_masses_plummer(env, cs):
    rng = np.random.default_rng(15)
    s = workloads.uniform_varied(20000, 16, target=60.0)
    s.h = (s.h * np.exp(rng.uniform(-1.2, 1.2, s.n))).astype(np.float32)
    m = rng.uniform(0.1, 3.0, s.n).astype(np.float32)
    _compare(s, _run(env, s, mass=m, cs=cs), mass=m, cs=cs)
    p = workloads.plummer(30000, 23, target=150.0)
    _compare(p, _run(env, p, leaf_bucket=128, cs=cs), cs=cs)


@pytest.mark.parametrize("cs", CS_OTHER)
def test_cluster_size_ties_and_lattice(env, cs):
    rng = np.random.default_rng(19)
    n = 2000
    base = rng.random((3, 30)).astype(np.float32)
    pick = rng.integers(0, 30, n)
    s = workloads.ParticleSystem("ties", base[0][pick].copy(), base[1][pick].copy(), base[2][pick].copy(),
                                 np.full(n, 0.05, np.float32), None, workloads.UNIT_BOX)
    _compare(s, _run(env, s, cs=cs), cs=cs)
    a = 0.125
    g = np.arange(8, dtype=np.float32) * np.float32(a)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    lat = workloads.ParticleSystem("lattice", X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy(),
                                   np.full(X.size, 0.13, np.float32), None, workloads.UNIT_BOX)
    _compare(lat, _run(env, lat, cs=cs), method="brute", cs=cs)


@pytest.mark.parametrize("cs", CS_OTHER)
def test_cluster_size_decoder(env, cs):
    sf, ctx, torch = env
    s = workloads.uniform_varied(9000, 45, target=120.0)
    for compress in (True, False):
        g = _run(env, s, compress, cs=cs)
        offs, j, m = sf.nlist_decode(ctx, g["nl"])
        ref = oracle.pipeline(s.x, s.y, s.z, s.h, s.box, None, cs, compress)
        np.testing.assert_array_equal(offs, ref["offs"])
        np.testing.assert_array_equal(j, ref["j"])
        np.testing.assert_array_equal(m, ref["mask"])


# Half lists (each pair once, j > i; the pass feeds both particles of a pair
# through atomics): list bytes bit-exact, counts exact, densities within the
# tolerance.
CS_ALL = [8, 4, 16]


@pytest.mark.parametrize("cs", CS_ALL)
@pytest.mark.parametrize("compress", [True, False])
def test_half_uniform_32k(env, cs, compress):
    s = workloads.make_config("uniform_32k")
    _compare(s, _run(env, s, compress, cs=cs, half=True), compress, cs=cs, half=True)


@pytest.mark.parametrize("cs", CS_ALL)
@pytest.mark.parametrize("n", [1, 2, 9, 63, 65, 1000, 4099])
def test_half_small_and_ragged(env, cs, n):
    s = workloads.uniform_varied(n, 3000 + n, target=40.0)
    _compare(s, _run(env, s, cs=cs, half=True), cs=cs, half=True)


@pytest.mark.parametrize("cs", CS_ALL)
def test_half_varied_masses_plummer_ties(env, cs):
    rng = np.random.default_rng(25)
    s = workloads.uniform_varied(20000, 26, target=60.0)
    s.h = (s.h * np.exp(rng.uniform(-1.2, 1.2, s.n))).astype(np.float32)
    m = rng.uniform(0.1, 3.0, s.n).astype(np.float32)
    _compare(s, _run(env, s, mass=m, cs=cs, half=True), mass=m, cs=cs, half=True)
    p = workloads.plummer(30000, 27, target=150.0)
    _compare(p, _run(env, p, leaf_bucket=128, cs=cs, half=True), cs=cs, half=True)
    n = 2000
    base = rng.random((3, 30)).astype(np.float32)
    pick = rng.integers(0, 30, n)
    t = workloads.ParticleSystem("ties", base[0][pick].copy(), base[1][pick].copy(), base[2][pick].copy(),
                                 np.full(n, 0.05, np.float32), None, workloads.UNIT_BOX)
    _compare(t, _run(env, t, cs=cs, half=True), cs=cs, half=True)


def test_half_matches_full_counts_and_density(env):
    s = workloads.uniform_varied(50000, 28, target=120.0)
    full = _run(env, s)
    half = _run(env, s, half=True)
    np.testing.assert_array_equal(half["nnb"], full["nnb"])
    rel = np.abs(half["rho"].astype(np.float64) - full["rho"]) / full["rho"]
    assert rel.max() <= RHO_RTOL
    assert half["nl"].used_bytes < 0.62 * full["nl"].used_bytes


def test_capacity_retry_gives_identical_list(env):
    sf, ctx, torch = env
    s = workloads.uniform_varied(10000, 45, target=100.0)
    x, y, z, h = (_dev(torch, a) for a in (s.x, s.y, s.z, s.h))
    keys, perm = sf.sfc_sort(ctx, x, y, z, s.box)
    xs, ys, zs, hs = sf.sfc_gather(ctx, perm, [x, y, z, h])
    bbox = sf.build_clusters(ctx, xs, ys, zs, hs)
    big = sf.build_nlist(ctx, keys, xs, ys, zs, hs, bbox)
    ref_pool = _u32(big.pool)[: big.used_bytes // 4].copy()
    # too small a pool and staging list: the library reports sizes, no retry
    tiny = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(sf.SfcnlError) as ei:
        sf.build_nlist(ctx, keys, xs, ys, zs, hs, bbox, max_j_per_sc=4, pool=tiny, grow=False)
    assert ei.value.code == -3
    # growing retry gives the identical list
    again = sf.build_nlist(ctx, keys, xs, ys, zs, hs, bbox, max_j_per_sc=4, pool=tiny)
    assert again.used_bytes == big.used_bytes
    np.testing.assert_array_equal(_u32(again.pool)[: again.used_bytes // 4], ref_pool)
    np.testing.assert_array_equal(_u32(again.sc_info), _u32(big.sc_info))


def test_bad_input_reported(env):
    sf, ctx, torch = env
    s = workloads.uniform_varied(2000, 46, target=30.0)
    for field, val, flag in (("x", np.nan, 1), ("h", -1.0, 2), ("h", np.inf, 2)):
        a = {k: getattr(s, k).copy() for k in ("x", "y", "z", "h")}
        a[field][123] = val
        x, y, z, h = (_dev(torch, a[k]) for k in ("x", "y", "z", "h"))
        with pytest.raises(sf.SfcnlError) as ei:
            pipe = sf.Pipeline(ctx, s.n, s.box)
            pipe.step(x, y, z, h)
            ctx.sync()
        assert ei.value.code == -2
    ctx.sync()  # latch cleared


def test_bad_box_rejected(env):
    sf, ctx, torch = env
    x = torch.zeros(10, device="cuda")
    with pytest.raises(sf.SfcnlError) as ei:
        sf.sfc_sort(ctx, x, x, x, (0.0, 0.0, 0.0, 1.0, 0.0, 1.0))
    assert ei.value.code == -1


def test_repeat_is_deterministic(env):
    s = workloads.uniform_varied(50000, 47, target=200.0)
    a = _run(env, s)
    b = _run(env, s)
    np.testing.assert_array_equal(a["pool"], b["pool"])
    np.testing.assert_array_equal(a["rho"], b["rho"])


@pytest.mark.slow
@pytest.mark.parametrize("half", [True, False])
def test_uniform_2m_sampled(env, half):
    """Full 2,097,152-particle workload in the benchmark's configuration
    (cluster size 8, leaf bucket 128, compressed; the benchmark times the half
    list): exact lists for sampled super-clusters (oracle brute force over all
    particles), exact counts and densities for all particles (oracle cell list)."""
    sf, ctx, torch = env
    s = workloads.make_config("uniform_2m_varied")
    g = _run(env, s, leaf_bucket=128, half=half)
    _say("gpu done; oracle keys and order")
    keys = oracle.hilbert_keys(s.x, s.y, s.z, s.box)
    perm = oracle.sfc_order(keys)
    np.testing.assert_array_equal(g["perm"], perm)
    xs, ys, zs, hs = s.x[perm], s.y[perm], s.z[perm], s.h[perm]
    nsc = (s.n + 63) // 64
    ids = np.unique(np.concatenate([[0, nsc - 1], np.random.default_rng(1).integers(0, nsc, 14)]))
    _say("oracle brute-force lists for %d super-clusters" % len(ids))
    so, sj, sm = oracle.cluster_list(xs, ys, zs, hs, 8, "brute", sc_ids=ids, half=half)
    _say("compare lists, then oracle densities")
    info = g["sc_info"]
    for k, sc in enumerate(ids):
        nj = int(info[sc, 1])
        words = g["pool"][info[sc, 0]:]
        j, m, used = oracle.decode_sc(words, nj, 8, True)
        np.testing.assert_array_equal(j, sj[so[k]:so[k + 1]])
        np.testing.assert_array_equal(m, sm[so[k]:so[k + 1]])
        np.testing.assert_array_equal(words[:used], oracle.encode_sc(sj[so[k]:so[k + 1]], sm[so[k]:so[k + 1]]))
    rho, nnb = oracle.density(xs, ys, zs, hs, None, "grid")
    np.testing.assert_array_equal(g["nnb"], nnb)
    rel = np.abs(g["rho"].astype(np.float64) - rho) / rho
    assert rel.max() <= RHO_RTOL, rel.max()
    # under max(h_i, h_j): ~190 j-clusters per super-cluster in the full list,
    # ~97 in the half list (each pair once)
    assert g["nl"].bytes_per_particle() < (2.4 if half else 4.25)


def test_staging_sized_by_total_length(env):
    """A Plummer sphere (radii for ~60 neighbours at the local density) whose
    40 central particles have radius 0.6: the super-clusters holding them list
    thousands of j-clusters (above 4,096), the others about a hundred. The
    staging list is sized by the total list length (every super-cluster's
    first 64-entry chunk plus shared chunks), so the build succeeds with
    staging room near the mean list length; every pool word equals the
    oracle's."""
    sf, ctx, torch = env
    s = workloads.plummer(40000, 78, target=60.0)
    r = np.sqrt(s.x.astype(np.float64) ** 2 + s.y ** 2 + s.z ** 2)
    a = 0.1
    dens = s.n * 3.0 / (4.0 * np.pi * a ** 3) * (1.0 + r ** 2 / a ** 2) ** -2.5
    s.h = ((3.0 * 60.0 / (4.0 * np.pi * dens)) ** (1.0 / 3.0)).astype(np.float32)
    core = np.argsort(r)[:40]
    s.h[core] = np.float32(0.6)
    x, y, z, h = (_dev(torch, a) for a in (s.x, s.y, s.z, s.h))
    keys, perm = sf.sfc_sort(ctx, x, y, z, s.box)
    xs, ys, zs, hs = sf.sfc_gather(ctx, perm, [x, y, z, h])
    bbox = sf.build_clusters(ctx, xs, ys, zs, hs)
    nl = sf.build_nlist(ctx, keys, xs, ys, zs, hs, bbox, max_j_per_sc=64)
    info = _u32(nl.sc_info)
    nj = info[:, 1].astype(np.int64)
    total = int(nj.sum())
    _say("longest list %d, total %d entries over %d super-clusters; max_j_per_sc grew to %d"
         % (nj.max(), total, nj.shape[0], nl.max_j_per_sc))
    assert nj.max() > 4096
    # staging entries (whole chunks per super-cluster on average) within 1.5x
    # of the entries the lists hold
    staging = nj.shape[0] * ((nl.max_j_per_sc + 63) // 64) * 64
    assert staging * 6 <= 1.5 * total * 6, (staging, total)
    xa, ya, za, ha = (t.cpu().numpy() for t in (xs, ys, zs, hs))
    offs, jj, mm = oracle.cluster_list(xa, ya, za, ha, 8, "grid")
    oinfo, opool = oracle.encode_all(offs, jj, mm, 8, True)
    np.testing.assert_array_equal(info, oinfo)
    np.testing.assert_array_equal(_u32(nl.pool)[: nl.used_bytes // 4], opool)


@pytest.mark.parametrize("half", [False, True])
def test_pass_waves_per_block(env, half):
    """The density pass's workgroup shape (1, 2 or 4 wavefronts per block, the
    autotuner's knob) changes no result: counts exact, full-list densities
    bit-identical, half-list densities within the atomics' summation order."""
    sf, ctx, torch = env
    s = workloads.uniform_varied(20011, 51, target=100.0)
    x, y, z, h = (_dev(torch, a) for a in (s.x, s.y, s.z, s.h))
    keys, perm = sf.sfc_sort(ctx, x, y, z, s.box)
    xs, ys, zs, hs = sf.sfc_gather(ctx, perm, [x, y, z, h])
    bbox = sf.build_clusters(ctx, xs, ys, zs, hs)
    nl = sf.build_nlist(ctx, keys, xs, ys, zs, hs, bbox, half=half)
    res = {}
    try:
        for w in (1, 2, 4):
            ctx.set_pass_waves(w)
            r, c = sf.nlist_pass(ctx, nl, xs, ys, zs, hs)
            res[w] = (r.cpu().numpy(), c.cpu().numpy())
    finally:
        ctx.set_pass_waves(1)
    for w in (2, 4):
        np.testing.assert_array_equal(res[w][1], res[1][1])
        if half:
            np.testing.assert_allclose(res[w][0], res[1][0], rtol=2e-6, atol=0)
        else:
            np.testing.assert_array_equal(res[w][0], res[1][0])
    with pytest.raises(sf.SfcnlError):
        ctx.set_pass_waves(3)


@pytest.mark.parametrize("cs", [4, 8, 16])
def test_cluster_boxes_unaligned_fields(env, cs):
    # fields 4 bytes off a 16-byte boundary take the per-particle loads, aligned
    # ones the vector loads: the boxes agree bit for bit, and with the oracle
    sf, ctx, torch = env
    n = 10_007
    _say("cluster boxes unaligned cs=%d n=%d" % (cs, n))
    s = workloads.uniform_varied(n, 5100 + cs, target=40.0)
    keys = oracle.hilbert_keys(s.x, s.y, s.z, s.box)
    order = np.argsort(keys, kind="stable")
    cols = [np.ascontiguousarray(a[order]) for a in (s.x, s.y, s.z, s.h)]
    big = [_dev(torch, np.concatenate([np.zeros(1, np.float32), c])) for c in cols]
    off = [b[1:] for b in big]  # storage offset 4 bytes
    ali = [_dev(torch, c) for c in cols]
    nc = (n + cs - 1) // cs
    b_off = torch.empty((nc, 8), dtype=torch.float32, device="cuda")
    b_ali = torch.empty((nc, 8), dtype=torch.float32, device="cuda")
    sf.build_clusters(ctx, *off, cs, b_off)
    sf.build_clusters(ctx, *ali, cs, b_ali)
    torch.cuda.synchronize()
    assert off[0].data_ptr() % 16 == 4 and ali[0].data_ptr() % 16 == 0
    assert torch.equal(b_off, b_ali)
    ref = oracle.cluster_bboxes(*cols, cs)
    got = b_ali.cpu().numpy()
    np.testing.assert_array_equal(got[:, :4], ref[:, :4])
    np.testing.assert_array_equal(got[:, 4:7], ref[:, 4:7])
