"""Lennard-Jones 12/6 + Coulomb pass (Sec. III benchmark) against the FP64
oracle, through the C ABI.

The list is built at the list radius (~200 neighbours) and the pass keeps the
pairs inside the interaction cutoff (~150), as with a Verlet buffer. Bar: per
particle and component |F_gpu - F_oracle| <= 1e-5 * sum_j |F_ij| (FP32 terms
of a few ulp each, summed over ~150 pairs in any order, stay far below it),
and the same for the energies against sum_j |U_ij| / 2. The oracle runs on the
generator's arrays in the generator's order; the GPU's SFC permutation is
first checked equal to the oracle's own.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2602_19873_amd import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5


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


def _holes(s, keep, seed):
    """The lattice with random atoms removed (ragged n, uneven clusters)."""
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(s.n, keep, replace=False))
    return workloads.ParticleSystem(s.name + "_holes", s.x[idx], s.y[idx], s.z[idx], s.h[idx], None, s.box,
                                    dict(s.meta), q=s.q[idx])


def _gpu(env, s, cs, half, compress, charges, energy, bucket=64):
    sf, ctx, torch = env
    _say("lj case n=%d cs=%d half=%d compress=%d charges=%d energy=%d" % (s.n, cs, half, compress, charges, energy))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    x, y, z, h, q = (dev(a) for a in (s.x, s.y, s.z, s.h, s.q))
    pipe = sf.Pipeline(ctx, s.n, s.box, compress, bucket, 512, with_mass=True, cluster_size=cs, half=half)
    nl = pipe.step(x, y, z, h, q)  # q rides along as the fifth gathered field
    xs, ys, zs, _, qs = pipe.sorted
    mt = s.meta
    f, e = sf.nlist_pass_lj(ctx, nl, xs, ys, zs, qs if charges else None, mt["eps"], mt["sigma"], mt["coulomb"],
                            mt["r_cut"], energy=energy)
    torch.cuda.synchronize()
    perm = pipe.perm.cpu().numpy().view(np.uint32).astype(np.int64)
    return perm, f.cpu().numpy().T.astype(np.float64), (None if e is None else e.cpu().numpy().astype(np.float64))


def _check(s, perm, f, e, charges, rows=None):
    ref_perm = oracle.sfc_order(oracle.hilbert_keys(s.x, s.y, s.z, s.box))
    np.testing.assert_array_equal(perm, ref_perm)
    mt = s.meta
    idx = np.arange(s.n) if rows is None else np.asarray(rows)
    ref = oracle.lj(s.x, s.y, s.z, s.q if charges else None, mt["eps"], mt["sigma"], mt["coulomb"], mt["r_cut"],
                    idx=idx)
    inv = np.empty(s.n, np.int64)
    inv[perm] = np.arange(s.n)
    g = f[inv[idx]]
    err = np.abs(g - ref["f"]).max(axis=1) / ref["scale"]
    assert np.all(np.isfinite(g))
    assert err.max() <= TOL, "force error %.3g at row %d" % (err.max(), int(err.argmax()))
    if e is not None:
        ge = e[inv[idx]]
        eerr = np.abs(ge - ref["e"]) / ref["escale"]
        assert eerr.max() <= TOL, "energy error %.3g" % eerr.max()
    return err.max()


@pytest.fixture(scope="module")
def lattices():
    s = workloads.lj_lattice(20, workloads.SEED_BASE + 60)
    return {"full": s, "holes": _holes(s, 7937, 61)}


CASES = [(cs, half, True, True, True) for cs in (8, 4, 16) for half in (False, True)] + \
        [(8, False, False, False, False), (8, True, False, False, True), (16, True, False, True, False)]


@pytest.mark.parametrize("which", ["full", "holes"])
@pytest.mark.parametrize("cs,half,compress,charges,energy", CASES)
def test_lj_matches_oracle(env, lattices, which, cs, half, compress, charges, energy):
    s = lattices[which]
    perm, f, e = _gpu(env, s, cs, half, compress, charges, energy)
    err = _check(s, perm, f, e, charges)
    _say("  max force error / scale %.2e" % err)


def test_lj_full_and_half_agree(env, lattices):
    s = lattices["holes"]
    _, f0, e0 = _gpu(env, s, 8, False, True, True, True)
    _, f1, e1 = _gpu(env, s, 8, True, True, True, True)
    ref = oracle.lj(s.x, s.y, s.z, s.q, s.meta["eps"], s.meta["sigma"], s.meta["coulomb"], s.meta["r_cut"])
    # both in SFC order; same particles
    assert np.all(np.abs(f0 - f1).max(axis=1) <= 2 * TOL * ref["scale"].max())


def test_lj_momentum_half_list(env, lattices):
    # Newton's third law on the device: the half list adds +-F of every pair
    s = lattices["full"]
    _, f, _ = _gpu(env, s, 8, True, True, True, False)
    ref = oracle.lj(s.x, s.y, s.z, s.q, s.meta["eps"], s.meta["sigma"], s.meta["coulomb"], s.meta["r_cut"])
    assert np.all(np.abs(f.sum(axis=0)) <= 1e-5 * ref["scale"].sum())


def test_lj_4m_sampled(env):
    # the benchmark size: 160^3 atoms, 2000 sampled rows against the oracle
    s = workloads.make_config("lj_4m")
    rows = np.random.default_rng(62).choice(s.n, 2000, replace=False)
    for half in (True, False):
        perm, f, e = _gpu(env, s, 8, half, True, True, True, bucket=128)
        err = _check(s, perm, f, e, True, rows)
        _say("  4m half=%d max force error / scale %.2e" % (half, err))
