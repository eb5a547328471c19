"""Training data and evaluation for the learned smoothing-length seed.

Training pairs come from the method itself: particles of the uniform
generator with per-particle radii get a perturbed starting radius h_prev; one
round of list build + pass gives their neighbour counts and the features, and
sfcnl_h_iterate drives them to convergence; the regression target is
log(h_converged / h_prev). Everything on the device runs in the library's
kernels; the host only draws the perturbation and forms the target.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import (CLUSTER_SIZE, build_clusters, build_nlist, h_iterate, hseed_features, nlist_pass, sfc_gather,
               sfc_sort)
from . import workloads


def box_edge(box) -> float:
    return float(max(box[1] - box[0], box[3] - box[2], box[5] - box[4]))


def sorted_system(ctx, s, h=None):
    """Uploads a system and puts it in SFC order: (keys, x, y, z, h)."""
    dev = torch.device("cuda:%d" % ctx.device)
    hh = s.h if h is None else h
    x, y, z, hd = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (s.x, s.y, s.z, hh))
    keys, perm = sfc_sort(ctx, x, y, z, s.box)
    xs, ys, zs, hs = sfc_gather(ctx, perm, [x, y, z, hd])
    return keys, xs, ys, zs, hs


def training_pairs(ctx, s, target: int, h_prev: np.ndarray, max_iters: int = 64, before_first: bool = False):
    """(features int16 bf16 bits [n, 8], targets float32 [n]) for one system.
    before_first: features without a count (the seed applied before the
    first round), so no list is built at h_prev."""
    keys, xs, ys, zs, hs = sorted_system(ctx, s, h_prev)
    if before_first:
        nnb = None
    else:
        bbox = build_clusters(ctx, xs, ys, zs, hs)
        nl = build_nlist(ctx, keys, xs, ys, zs, hs, bbox)
        _, nnb = nlist_pass(ctx, nl, xs, ys, zs, hs)
    feat = hseed_features(ctx, keys, xs, ys, zs, hs, nnb, box_edge(s.box), target)
    hc = hs.clone()
    res = h_iterate(ctx, keys, xs, ys, zs, hc, target=target, tol=1, max_iters=max_iters)
    if not res.converged:
        raise RuntimeError("training system did not converge")
    d = np.log(hc.cpu().numpy().astype(np.float64) / hs.cpu().numpy().astype(np.float64)).astype(np.float32)
    return feat, torch.from_numpy(d).to(feat.device)


def training_set(ctx, n_total: int = 1 << 20, targets=(50, 100, 150, 200), spread: float = 4.0, seed: int = 7):
    """Pairs from the uniform generator with radii r_c U(0.8, 1.2) (the 2M
    benchmark's generator), n_total particles split over the targets; the
    starting radius is the generator's radius times a log-uniform factor in
    [1/spread, spread]."""
    feats, ds = [], []
    per = n_total // len(targets)
    for k, T in enumerate(targets):
        s = workloads.uniform_varied(per, workloads.SEED_BASE + 2 + 10 * k, target=T)
        rng = np.random.default_rng(seed * 1000 + k)
        hp = (s.h * np.exp(rng.uniform(-math.log(spread), math.log(spread), s.n))).astype(np.float32)
        f, d = training_pairs(ctx, s, T, hp)
        feats.append(f)
        ds.append(d)
    return torch.cat(feats), torch.cat(ds)


def mixed_training_set(ctx, target: int = 150, count: int = 16, lo: float = 1e4, hi: float = 2e5,
                       spread: float = 2.0, seed: int = 11, before_first: bool = True):
    """Pairs from the batch generators (uniform cube and Plummer sphere,
    alternating; sizes log-uniform in [lo, hi]) with seeds disjoint from the
    benchmark batch's; the starting radius is the generator's mean-density
    radius times a log-uniform factor in [1/spread, spread]."""
    feats, ds = [], []
    for k in range(count):
        rng = np.random.default_rng(seed * 7919 + k)
        nk = int(round(10.0 ** rng.uniform(math.log10(lo), math.log10(hi))))
        gseed = seed * 100003 + k
        s = workloads.uniform_global(nk, gseed, target) if k % 2 == 0 else workloads.plummer(nk, gseed, target=target)
        hp = (s.h * np.exp(rng.uniform(-math.log(spread), math.log(spread), s.n))).astype(np.float32)
        f, d = training_pairs(ctx, s, target, hp, before_first=before_first)
        feats.append(f)
        ds.append(d)
    return torch.cat(feats), torch.cat(ds)


def iterate(ctx, s, target: int, mlp_params=None, bufs=None, max_iters: int = 64):
    """Runs the iteration on a system from its own radii; returns the result,
    the final SFC-ordered arrays and the buffers for reuse."""
    keys, xs, ys, zs, hs = sorted_system(ctx, s)
    kw = dict(bufs or {})
    res = h_iterate(ctx, keys, xs, ys, zs, hs, target=target, tol=1, max_iters=max_iters, mlp_params=mlp_params,
                    box_edge=box_edge(s.box), **kw)
    return res, (keys, xs, ys, zs, hs)
