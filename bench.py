#!/usr/bin/env python
"""Throughput of the SFC cluster neighbour list: list build + density pass.

One step = the whole path over one system already resident in HBM:
Hilbert keys + stable radix sort, gather into SFC order, cluster boxes,
octree + traversal + compressed encoding, decode + SPH density pass.

Prints one JSON line (rank 0, one GPU). Per-kernel durations come from HIP
events the library records on its own stream inside the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "nlist build + density pass Mparticles/s at 1 GPU; bytes/particle; % HBM roofline"

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3      # 256 CU x 2.4 GHz x 128 FP32 lanes (dual-issue) x 2 (FMA)

# Algorithmic work, per unit (stated also in the design doc):
#   HBM stages: bytes per particle the stage must move at minimum.
#   ALU stages: FP32 flops (an FMA counts 2) per particle-pair test.
BYTES_PER_PARTICLE = {
    "keys": 12 + 8 + 4,            # read x, y, z; write key and index (the first pass's histogram on the way)
    "sort": 3 * (12 + 12) + 2 * 8 + 12,  # 3 prefix passes: read + write key/index, two histogram reads of
                                         # the keys; the local sort reads key/index once (rewrites ~1.5 %)
    "gather": 4 + 4 * (4 + 4),     # read perm; read + write x, y, z, h
    "clusters": 16 + 4,            # read x, y, z, h; write 32 B per 8-particle cluster
    "octree": 8 + 4,               # read the sorted keys and the cluster boxes (nodes are ~1/16 of that)
    "traverse": 16,                # read x, y, z, h of the own super-cluster (j-data from L2)
    "pass": 16 + 8,                # read x, y, z, h; write rho, nnb (plus the list, counted per byte)
}
# Counted tests and evaluations: 64 per set mask bit of the final list (the 8x8
# tiles that establish the list in the build and that the pass evaluates).
FLOPS_PER_TEST = 9      # dx, dy, dz (3); dx*dx (1); two fma (4); compares are not counted
FLOPS_PER_PAIR = 17     # dx, dy, dz (3); d2 (5); sqrt (1); q (1); spline piece (5); m*W, += (2)
FLOPS_PER_PAIR_HALF = 25  # one distance (9), then q, spline piece, m*W, += for both particles (2 x 8)


# Lennard-Jones + Coulomb pass, per evaluated tile pair: dx, dy, dz (3); d2 (3);
# cutoff compare (1); 1/r^2, (sigma^2/r^2)^3, 24 eps (2 s6 - 1) s6 / r^2 (7);
# 1/r, k q_i q_j / r, fma into the force factor (4); select (1); three fma into
# the force sums (3). The half list adds three products and three sums for j.
LJ_FLOPS_PER_PAIR = 22
LJ_FLOPS_PER_PAIR_HALF = 28


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name):
    from paper_2602_19873_amd import workloads
    return workloads.make_config(name)


def list_stats(sf, ctx, nl):
    """Bytes per particle split, and the pair work the list fixes."""
    import numpy as np
    offs, j, m = sf.nlist_decode(ctx, nl)
    mm = m.astype(np.uint16)
    pc = int(np.unpackbits(mm.view(np.uint8)).sum()) if m.size else 0
    nj = np.diff(offs)
    n = nl.n
    mask_bytes = float(((nj + 3) // 4 * 4).sum())
    return {
        "bytes_per_particle": nl.bytes_per_particle(),
        "bytes_headers_pp": 8.0 * nl.n_sc / n,
        "bytes_masks_pp": mask_bytes / n,
        "bytes_indices_pp": (nl.used_bytes - mask_bytes) / n,
        "entries": int(nj.sum()),
        "mean_nj": float(nj.mean()) if nj.size else 0.0,
        "max_nj": int(nj.max()) if nj.size else 0,
        "tile_pairs": int(pc) * nl.cluster_size ** 2,   # cs x cs pair tests per set mask bit
        "half": bool(nl.half),
    }


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(s, runs=3, one_thread_n=262144):
    """The oracle, as it stands, on the timed workload itself (keys, stable
    order, cell-list cluster list, encoding, FP64 density): the median of
    `runs` runs on all host threads, and one run on one thread over a bounded
    sample of the same generator (same neighbour count, fewer particles)."""
    import statistics
    import oracle
    from paper_2602_19873_amd import workloads
    oracle.build()
    nthreads = oracle.num_threads()
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        oracle.pipeline(s.x, s.y, s.z, s.h, s.box)
        ts.append(time.perf_counter() - t0)
    dt = statistics.median(ts)
    small = workloads.uniform_varied(one_thread_n, workloads.SEED_BASE + 2, target=200.0)
    oracle.set_num_threads(1)
    t0 = time.perf_counter()
    oracle.pipeline(small.x, small.y, small.z, small.h, small.box)
    dt1 = time.perf_counter() - t0
    oracle.set_num_threads(nthreads)
    return {"value": s.n / dt / 1e6, "unit": "Mparticles/s", "cores": nthreads, "kind": "oracle",
            "sample": "the full timed workload (%s, N=%d): the whole oracle path (Hilbert keys, stable sort, "
                      "cell-list cluster list, nibble encoding, FP64 density), median of %d runs on %d threads "
                      "(%.1f s); one thread: the same generator at N=%d"
                      % (s.name, s.n, runs, nthreads, dt, one_thread_n),
            "seconds": dt, "runs_s": ts, "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "one_thread": {"value": one_thread_n / dt1 / 1e6, "unit": "Mparticles/s", "n": one_thread_n,
                           "seconds": dt1}}


def source_sha(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:12]


# Kernels of each stage of a step (for the counter-byte figures).
STAGE_KERNELS = {
    "keys": ["k_keys_hist"],
    "sort": ["k_hist", "k_digit_scan", "k_scatter", "k_local_sort"],
    "gather": ["k_pack4", "k_gather4"],
    "clusters": ["k_cluster_bbox"],
    "octree": ["k_leaf_level", "k_emit_nodes", "k_node_range", "k_children", "k_box_levels",
               "k_node_slots"],
}


def read_counters(n):
    """HBM bytes per launch of each kernel from the committed counter summary
    (lines `traffic kernel=... source=... source_sha=... n=... bytes_per_launch=...
    launches_per_step=...`); a kernel whose source changed since the counters
    were taken is left out."""
    path = os.path.join(ROOT, "profiles", "counters_uniform_2m.txt")
    out = {}
    if not os.path.exists(path):
        return out
    with open(path) as f:
        for line in f:
            if not line.startswith("traffic "):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[1:])
            if int(kv["n"]) != n:
                continue
            src = os.path.join(ROOT, "paper_2602_19873_amd", "csrc", kv["source"])
            if not os.path.exists(src) or kv["source_sha"] != source_sha(src):
                continue
            out[kv["kernel"]] = (float(kv["bytes_per_launch"]), float(kv.get("launches_per_step", "1")))
    return out


def read_traffic(kernel, n):
    """HBM bytes per launch of `kernel` (None if not measured for its current source)."""
    rec = read_counters(n).get(kernel.replace(" ", ""))
    return None if rec is None else rec[0]


def _hiter_system(args, name):
    """The 8,388,608-particle 1/r sphere from the plain global mean-density
    radius (or the analytic-density seed), or the uniform generator of the
    2M benchmark at the same size with starting radii off by a log-uniform
    factor in [1/spread, spread] (the learned seed's training distribution)."""
    import math
    import numpy as np
    from paper_2602_19873_amd import workloads
    T = args.target
    n = args.n or 8388608
    if name == "sphere":
        return workloads.evrard_sphere(n, workloads.SEED_BASE + 3, target=T, seed_h=args.seed_h)
    s = workloads.uniform_varied(n, workloads.SEED_BASE + 4, target=T)
    rng = np.random.default_rng(workloads.SEED_BASE + 5)
    sp = args.train_spread
    s.h = (s.h * np.exp(rng.uniform(-math.log(sp), math.log(sp), n))).astype(np.float32)
    s.name = "uniform_varied_8m_spread%g" % sp
    return s


def _time_hiter(args, sf, torch, ctx, s, params=None):
    """Median time of `steps` runs of the iteration from the starting radii;
    the SFC order is computed once outside the timed region (positions are
    fixed)."""
    from paper_2602_19873_amd import hseed
    T = args.target
    dev = torch.device("cuda:0")
    x, y, z, h = (torch.from_numpy(a).to(dev) for a in (s.x, s.y, s.z, s.h))
    keys, perm = sf.sfc_sort(ctx, x, y, z, s.box)
    xs, ys, zs, h0 = sf.sfc_gather(ctx, perm, [x, y, z, h])
    del x, y, z, h, perm
    hw = torch.empty_like(h0)
    bufs = {}
    if params is not None:
        bufs.update(mlp_params=params, box_edge=hseed.box_edge(s.box))
    times, res = [], None
    for rep in range(args.warmup + args.steps):
        hw.copy_(h0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = sf.h_iterate(ctx, keys, xs, ys, zs, hw, target=T, tol=1, max_iters=64, half=bool(args.half),
                           recount=args.recount, **bufs)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        bufs.update(ws=res.nl.ws, pool=res.nl.pool, max_j_per_sc=res.nl.max_j_per_sc)
        if rep >= args.warmup:
            times.append(dt)
        log("  rep %d: %d rounds (mean %.2f), %.1f ms, converged=%s" % (rep, res.iters, res.mean_rounds(), dt * 1e3,
                                                                      res.converged))
    if not res.converged:
        raise RuntimeError("%s did not converge" % s.name)
    t = sorted(times)[len(times) // 2]
    worst = int((res.nnb[:s.n].long() - T).abs().max().item())
    out = {"ms": t * 1e3, "mparticles_per_s": s.n / t / 1e6, "rounds": res.iters,
           "mean_rounds": res.mean_rounds(), "ms_per_round": t * 1e3 / res.iters, "max_abs_dev": worst}
    del keys, xs, ys, zs, h0, hw, res, bufs
    torch.cuda.empty_cache()
    return out


def run_hiter(args, sf, torch, ctx):
    """Time to drive every particle to target +- 1 own-radius neighbours by
    list rebuilds: the 1/r sphere from the plain starting guess, and with
    --mlp 1 also the learned seed (trained on converged pairs of the 2M
    benchmark's generator at 1,048,576 particles; training is a one-off
    outside the timed region) against the plain rule, on the sphere and on
    the training generator at the same size."""
    from paper_2602_19873_amd import hseed
    T = args.target
    names = ("sphere", "uniform") if args.mlp else ("sphere",)
    params, train = None, None
    if args.mlp:
        log("training the seed on %d pairs of the uniform generator (spread x%g)" % (args.train_n, args.train_spread))
        t0 = time.perf_counter()
        feat, d = hseed.training_set(ctx, n_total=args.train_n, targets=(T,), spread=args.train_spread)
        params, losses = sf.mlp_train(ctx, feat, d, epochs=args.train_epochs, batch=4096)
        torch.cuda.synchronize()
        train = {"pairs": int(feat.shape[0]), "seconds": time.perf_counter() - t0, "loss_first": losses[0],
                 "loss_last": losses[-1], "target_variance": float(torch.var(d).item()),
                 "generator": "uniform, r_c U(0.8, 1.2), start x e^U(-ln s, ln s), s = %g" % args.train_spread}
        log("trained: loss %.4f -> %.4f (variance %.4f) in %.1f s" % (losses[0], losses[-1],
                                                                      train["target_variance"], train["seconds"]))
        del feat, d
    results = {}
    for name in names:
        s = _hiter_system(args, name)
        log("h-iteration: %s n=%d target=%d" % (s.name, s.n, T))
        log(" plain rule")
        r = {"plain": _time_hiter(args, sf, torch, ctx, s)}
        if params is not None:
            log(" learned seed")
            r["seeded"] = _time_hiter(args, sf, torch, ctx, s, params)
            r["speedup"] = r["plain"]["ms"] / r["seeded"]["ms"]
        r["workload"] = s.name
        r["n"] = s.n
        results[name] = r
    main = results["sphere"]["seeded" if args.mlp else "plain"]
    out = {"metric": "h-iteration to target +- 1 neighbours, Mparticles/s (N / time to convergence)",
           "value": main["mparticles_per_s"], "unit": "Mparticles/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": main["ms"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": results["sphere"]["workload"], "n": results["sphere"]["n"], "target": T, "tol": 1,
                      "seed_h": args.seed_h, "cluster_size": 8, "learned_seed": bool(args.mlp),
                      "list": "half (each pair once, j > i)" if args.half else "full"},
           "systems": results}
    if train:
        out["seed_training"] = train
    return out


def run_batch(args, sf, torch, ctx):
    """Batch of independent systems (sizes log-uniform in [1e4, 1e6], uniform
    cube and Plummer sphere alternating), every particle driven to target +- 1
    own-radius neighbours from the plain starting guess (each system's
    mean-density radius). Compared: the plain iteration run per system, one
    call after another, against the batched iteration (one set of launches
    per round over all systems, replayed from a HIP graph) with the learned
    seed applied before the first round and the autotuned leaf bucket.
    Positions are fixed, so the SFC order is computed outside the timed
    region; the seed's training is a one-off outside it too."""
    import numpy as np
    from paper_2602_19873_amd import autotune, hseed, workloads
    T = args.target
    systems = workloads.batch_systems(args.nsys, target=T)
    counts = [s.n for s in systems]
    ntot = sum(counts)
    log("batch: %d systems, %d particles (%d .. %d), target %d" % (len(systems), ntot, min(counts), max(counts), T))
    dev = torch.device("cuda:0")
    singles = [hseed.sorted_system(ctx, s) for s in systems]
    h0s = [a[4].clone() for a in singles]
    b = sf.Batch(ctx, counts, [s.box for s in systems])
    cat = lambda f: torch.from_numpy(np.ascontiguousarray(np.concatenate([getattr(s, f) for s in systems]))).to(dev)
    keys, perm = sf.batch_sort(ctx, b, cat("x"), cat("y"), cat("z"))
    xs, ys, zs, hb = sf.batch_gather(ctx, b, perm, [cat("x"), cat("y"), cat("z"), cat("h")])
    h0b = hb.clone()
    real = torch.zeros(b.n_pad, dtype=torch.bool, device=dev)
    for k in range(b.nsys):
        real[int(b.pbase[k]):int(b.pbase[k]) + counts[k]] = True
    torch.cuda.synchronize()

    log("training the seed (before-first-round features)")
    t0 = time.perf_counter()
    feat, d = hseed.mixed_training_set(ctx, T, count=args.train_systems, before_first=True)
    params, losses = sf.mlp_train(ctx, feat, d, epochs=args.train_epochs, batch=4096)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    log("trained on %d pairs in %.1f s: loss %.4f -> %.4f (target variance %.4f)" %
        (feat.shape[0], train_s, losses[0], losses[-1], float(torch.var(d).item())))

    def worst_dev(nnb_list):
        return max(int((n_.long() - T).abs().max().item()) for n_ in nnb_list if n_.numel())

    single_bufs = [dict() for _ in systems]

    def plain_per_system(seeded):
        rounds, nnbs = [], []
        for k, (a, h0) in enumerate(zip(singles, h0s)):
            keys_k, x_k, y_k, z_k, h_k = a
            h_k.copy_(h0)
            kw = dict(single_bufs[k])
            if seeded:
                kw.update(mlp_params=params, box_edge=hseed.box_edge(systems[k].box),
                          seed_mode=sf.SEED_BEFORE_FIRST)
            res = sf.h_iterate(ctx, keys_k, x_k, y_k, z_k, h_k, target=T, tol=1, max_iters=64, half=bool(args.half),
                               recount=args.recount, **kw)
            single_bufs[k] = dict(ws=res.nl.ws, pool=res.nl.pool, max_j_per_sc=res.nl.max_j_per_sc)
            if not res.converged:
                raise RuntimeError("system %d did not converge" % k)
            rounds.append(res.iters)
            nnbs.append(res.nnb[:counts[k]])
        return rounds, nnbs

    batch_bufs = {}
    tuned = {"leaf_bucket": 128, "cluster_size": 8}

    def batched(seeded, use_graph=True):
        hb.copy_(h0b)
        kw = dict(mlp_params=params, seed_mode=sf.SEED_BEFORE_FIRST) if seeded else {}
        res = sf.batch_h_iterate(ctx, b, keys, xs, ys, zs, hb, target=T, tol=1, max_iters=64, use_graph=use_graph,
                                 leaf_bucket=tuned["leaf_bucket"], cluster_size=tuned["cluster_size"],
                                 half=bool(args.half), bufs=batch_bufs, recount=args.recount, **kw)
        if not res.converged:
            raise RuntimeError("batch did not converge")
        return res.sys_rounds.tolist(), [res.nnb[real]]

    def timed(fn, *a):
        ts, out = [], None
        for rep in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn(*a)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if rep >= args.warmup:
                ts.append(dt)
            log("  rep %d: %.1f ms, max rounds %d" % (rep, dt * 1e3, max(out[0])))
        ts.sort()
        t = ts[len(ts) // 2]
        return {"ms": t * 1e3, "mparticles_per_s": ntot / t / 1e6, "max_rounds": int(max(out[0])),
                "mean_system_rounds": float(np.mean(out[0])), "max_abs_dev": worst_dev(out[1])}

    log("plain iteration, per system")
    plain = timed(plain_per_system, False)
    log("batched seeded iteration: warm-up run, then leaf-bucket autotune at the converged radii")
    batched(True)
    tuned = autotune.tune_batch(ctx, b, keys, xs, ys, zs, hb, tag="batch%d_t%d" % (b.nsys, T), use_cache=False,
                                half=bool(args.half))
    log("autotune: %s" % tuned)
    log("batched seeded iteration (graph)")
    best = timed(batched, True)
    log("batched plain iteration (graph)")
    bplain = timed(batched, False)
    log("seeded iteration, per system")
    sseed = timed(plain_per_system, True)
    out = {"metric": "h-iteration of a %d-system batch to target +- 1 neighbours, Mparticles/s "
                     "(total N / time to convergence)" % b.nsys,
           "value": best["mparticles_per_s"], "unit": "Mparticles/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": best["ms"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "batch_%d_uniform_plummer" % b.nsys, "n_total": ntot, "n_padded": b.n_pad,
                      "sizes": "log-uniform [1e4, 1e6]", "target": T, "tol": 1,
                      "cluster_size": tuned["cluster_size"], "leaf_bucket": tuned["leaf_bucket"],
                      "list": "half (each pair once, j > i)" if args.half else "full"},
           "batched_seeded_graph": best, "plain_per_system": plain, "batched_plain_graph": bplain,
           "seeded_per_system": sseed, "speedup_vs_plain_per_system": plain["ms"] / best["ms"],
           "autotune": tuned, "seed_training": {"pairs": int(feat.shape[0]), "seconds": train_s,
                                                "loss_first": losses[0], "loss_last": losses[-1]}}
    return out


def run_lj(args, sf, torch, ctx):
    """The Lennard-Jones benchmark of Sec. III: a near-uniform box of 160^3
    atoms, the list built once at the radius holding ~200 neighbours and the
    12/6 Lennard-Jones + Coulomb forces evaluated inside the ~150-neighbour
    cutoff (a Verlet buffer). Times the list build (keys to encode) and the
    force pass separately for every cluster size, list form and compression;
    the JSON line reports the configuration given by the flags."""
    import numpy as np
    from paper_2602_19873_amd import workloads
    s = workloads.make_config("lj_4m", args.n or None)
    n, mt = s.n, s.meta
    log("lj: %s n=%d r_list=%.5f r_cut=%.5f" % (s.name, n, mt["r_list"], mt["r_cut"]))
    dev = torch.device("cuda:0")
    x, y, z, h, q = (torch.from_numpy(a).to(dev) for a in (s.x, s.y, s.z, s.h, s.q))
    main_cfg = (args.cluster_size, bool(args.compress), bool(args.half))
    period = (1.0, 1.0, 1.0) if args.periodic else None  # the lattice fills the unit box
    cfgs = [(cs, c, hf) for cs in (8, 4, 16) for hf in (True, False) for c in (True, False)] if args.sweep else []
    if main_cfg not in cfgs:
        cfgs.append(main_cfg)
    sweep, main = {}, None
    for cs, comp, hf in cfgs:
        pipe = sf.Pipeline(ctx, n, s.box, compress=comp, leaf_bucket=args.leaf_bucket, cluster_size=cs, half=hf,
                           max_j_per_sc=256, with_mass=True, period=period)
        for _ in range(max(args.warmup, 1)):
            pipe.step(x, y, z, h, q, density=False)
        torch.cuda.synchronize()
        ctx.profile_begin(args.steps)
        for _ in range(args.steps):
            pipe.step(x, y, z, h, q, density=False)
        prof_build = ctx.profile_end()
        nl = pipe.nl
        xs, ys, zs, _, qs = pipe.sorted
        f = ctx.empty((3, n), torch.float32)
        for _ in range(max(args.warmup, 1)):
            sf.nlist_pass_lj(ctx, nl, xs, ys, zs, qs, mt["eps"], mt["sigma"], mt["coulomb"], mt["r_cut"], f=f)
        torch.cuda.synchronize()
        ctx.profile_begin(args.steps)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            sf.nlist_pass_lj(ctx, nl, xs, ys, zs, qs, mt["eps"], mt["sigma"], mt["coulomb"], mt["r_cut"], f=f)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / args.steps
        prof_pass = ctx.profile_end()
        build_ms = sum(ms / c for k, (ms, c) in prof_build.items() if c and k != "pass")
        pass_ms = prof_pass["pass"][0] / prof_pass["pass"][1]
        st = list_stats(sf, ctx, nl)
        fl = LJ_FLOPS_PER_PAIR_HALF if hf else LJ_FLOPS_PER_PAIR
        tf = st["tile_pairs"] * fl / (pass_ms * 1e-3) / 1e12
        key = "cs%d_%s_%s" % (cs, "half" if hf else "full", "nibble" if comp else "plain")
        rec = {"build_ms": build_ms, "pass_ms": pass_ms, "pass_wall_ms": wall, "build_over_pass": build_ms / pass_ms,
               "bytes_per_particle": st["bytes_per_particle"], "tile_pairs_per_particle": st["tile_pairs"] / n,
               "pass_tflops": tf, "build_stages_ms": {k: ms / c for k, (ms, c) in prof_build.items() if c}}
        sweep[key] = rec
        log("%-22s build %.3f ms  pass %.3f ms  (%.2fx)  %.3f B/p  %.0f tile pairs/p  %.1f TFLOP/s"
            % (key, build_ms, pass_ms, build_ms / pass_ms, st["bytes_per_particle"], st["tile_pairs"] / n, tf))
        if (cs, comp, hf) == main_cfg:
            main = (key, rec, st)
        del pipe, nl, f
        torch.cuda.empty_cache()
    key, rec, st = main
    cs, comp, hf = main_cfg
    hb = "true" if hf else "false"
    kern = "k_pass_lj%s<%d, %s, true, false, %s>" % ("_half" if hf else "", cs, "true" if comp else "false",
                                                     "true" if period else "false")
    out = {
        "metric": "Lennard-Jones 12/6 + Coulomb force pass over the compressed cluster list, Mparticles/s",
        "value": n / (rec["pass_ms"] * 1e-3) / 1e6, "unit": "Mparticles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": rec["pass_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": s.name, "n": n, "cluster_size": cs, "compress": comp, "leaf_bucket": args.leaf_bucket,
                   "list": "half (each pair once, j > i)" if hf else "full", "list_neighbours": 200,
                   "cutoff_neighbours": 150, "charges": "rock salt +-1/2", "energy": False,
                   "boundaries": "periodic (minimum images)" if period else "open"},
        "build_ms": rec["build_ms"], "build_over_pass": rec["build_over_pass"],
        "bytes_per_particle": rec["bytes_per_particle"], "list": st,
        "roofline": {"kernel": kern, "bound": "alu", "achieved": rec["pass_tflops"], "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": rec["pass_tflops"] / FP32_PEAK_TFLOPS, "traffic": None,
                     "avg_ms": rec["pass_ms"]},
        "sweep": sweep,
    }
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        rows = np.arange(n)
        t0 = time.perf_counter()
        oracle.lj(s.x, s.y, s.z, s.q, mt["eps"], mt["sigma"], mt["coulomb"], mt["r_cut"], idx=rows)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": rows.size / dt / 1e6, "unit": "Mparticles/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "seconds": dt,
                               "sample": "FP64 Lennard-Jones + Coulomb forces of all %d atoms of the box (cell "
                                         "list, no list build), %.1f s" % (n, dt)}
        if period:
            t0 = time.perf_counter()
            oracle.lj(s.x, s.y, s.z, s.q, mt["eps"], mt["sigma"], mt["coulomb"], mt["r_cut"], period=period)
            out["cpu_baseline"]["periodic_seconds"] = time.perf_counter() - t0
    print(json.dumps(out), flush=True)


def run_rows(args, sf, torch, ctx):
    """The compressed 1x1 list (the paper's future-work combination of the
    index compression with a full neighbour list) against the cluster lists
    on the benchmark workload: list sizes, build times and density-pass times
    of the full and half cluster lists and of the rows (compressed and raw)."""
    s = make_workload(args.workload)
    n = s.n
    dev = torch.device("cuda:0")
    x, y, z, h = (torch.from_numpy(a).to(dev) for a in (s.x, s.y, s.z, s.h))
    log("rows: %s n=%d" % (s.name, n))
    res = {}

    def timed(fn, steps):
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(steps):
            fn()
        e1.record(ctx.stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / steps

    cs = args.cluster_size
    for half in (True, False):
        pipe = sf.Pipeline(ctx, n, s.box, compress=True, leaf_bucket=args.leaf_bucket, cluster_size=cs, half=half)
        build = timed(lambda: pipe.step(x, y, z, h, density=False), args.steps)
        xs, ys, zs, hs = pipe.sorted[:4]
        nl = pipe.nl
        ps = timed(lambda: sf.nlist_pass(ctx, nl, xs, ys, zs, hs, rho=pipe.rho, nnb=pipe.nnb), args.steps)
        key = "cluster_%s" % ("half" if half else "full")
        res[key] = {"bytes_per_particle": nl.bytes_per_particle(), "build_ms": build, "pass_ms": ps}
        log("%-14s %.3f B/p  build %.3f ms  pass %.3f ms" % (key, nl.bytes_per_particle(), build, ps))
        if not half:
            for comp in (True, False):
                box = {}

                def mk():
                    box["rl"] = sf.build_rows(ctx, nl, xs, ys, zs, hs, compress=comp, pool=box.get("pool"),
                                              ws=box.get("ws"))
                    box["pool"], box["ws"] = box["rl"].pool, box["rl"].ws
                rb = timed(mk, args.steps)
                rl = box["rl"]
                rp = timed(lambda: sf.rows_pass(ctx, rl, xs, ys, zs, hs, rho=pipe.rho, nnb=pipe.nnb), args.steps)
                key = "rows_%s" % ("nibble" if comp else "raw")
                res[key] = {"bytes_per_particle": rl.bytes_per_particle(), "rows_from_cluster_list_ms": rb,
                            "build_ms": build + rb, "pass_ms": rp}
                log("%-14s %.3f B/p  rows %.3f ms (+ cluster build)  pass %.3f ms" % (key, rl.bytes_per_particle(),
                                                                                    rb, rp))
                del box
        del pipe, nl
        torch.cuda.empty_cache()
    best = res["rows_nibble"]
    out = {"metric": "compressed 1x1 list: density pass Mparticles/s (and list bytes/particle)",
           "value": n / (best["pass_ms"] * 1e-3) / 1e6, "unit": "Mparticles/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": best["pass_ms"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": args.workload, "n": n, "cluster_size": cs, "leaf_bucket": args.leaf_bucket},
           "lists": res}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform_2m_varied")
    ap.add_argument("--compress", type=int, default=1)
    ap.add_argument("--leaf-bucket", type=int, default=128)
    ap.add_argument("--cluster-size", type=int, default=8)
    ap.add_argument("--half", type=int, default=1, help="1: half list (each pair once), 0: full list")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="after warm-up, copy this many MiB once (counter calibration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the 32k and 8M build + pass figures, the 8M "
                                                             "h-iteration and the 64-system batch")
    ap.add_argument("--mode", choices=["step", "hiter", "batch", "lj", "rows"], default="step")
    ap.add_argument("--target", type=int, default=0, help="neighbour target (hiter 100, batch 150)")
    ap.add_argument("--nsys", type=int, default=64)
    ap.add_argument("--train-systems", type=int, default=16)
    ap.add_argument("--train-epochs", type=int, default=20)
    ap.add_argument("--seed-h", choices=["global", "analytic"], default="global")
    ap.add_argument("--mlp", type=int, default=0, help="hiter mode: also train and time the learned seed")
    ap.add_argument("--train-n", type=int, default=1 << 20, help="hiter --mlp: training particles")
    ap.add_argument("--train-spread", type=float, default=4.0, help="hiter --mlp: starting-radius spread")
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--recount", type=int, default=0, help="hiter/batch: rounds after the first recount by "
                                                            "0 automatic choice, 1 lists, 2 one wave per moved particle")
    ap.add_argument("--periodic", type=int, default=0, help="lj mode: periodic box (the lattice fills it)")
    ap.add_argument("--sweep", type=int, default=1, help="lj mode: also time every cluster size, list form and "
                                                          "compression (0: only the flagged configuration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the path runs on a single MI355X and no multi-GPU "
              "sharding is built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2602_19873_amd as sf

    if args.mode in ("hiter", "batch", "lj", "rows"):
        torch.cuda.set_device(0)
        ctx = sf.Context(0)
        if args.mode == "lj":
            run_lj(args, sf, torch, ctx)
        elif args.mode == "rows":
            run_rows(args, sf, torch, ctx)
        elif args.mode == "hiter":
            args.target = args.target or 100
            print(json.dumps(run_hiter(args, sf, torch, ctx)), flush=True)
        else:
            args.target = args.target or 150
            print(json.dumps(run_batch(args, sf, torch, ctx)), flush=True)
        ctx.close()
        return

    torch.cuda.set_device(0)
    ctx = sf.Context(0)
    run_step(args, sf, torch, ctx)
    ctx.close()


def time_steps(sf, torch, ctx, s, args, steps, warmup, copy_probe=0):
    """Times `steps` whole-path steps (keys to density pass) of system s on the
    library's stream; returns (ms per step, per-stage event times, list
    statistics)."""
    dev = torch.device("cuda:0")
    x, y, z, h = (torch.from_numpy(a).to(dev) for a in (s.x, s.y, s.z, s.h))
    pipe = sf.Pipeline(ctx, s.n, s.box, compress=bool(args.compress), leaf_bucket=args.leaf_bucket,
                       cluster_size=args.cluster_size, half=bool(args.half), max_j_per_sc=128 if args.half else 256)
    for _ in range(max(warmup, 1)):
        pipe.step(x, y, z, h)
    torch.cuda.synchronize()
    if copy_probe:
        src = torch.empty(copy_probe << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy probe: %d MiB" % copy_probe)
    # the per-stage breakdown first: as many steps as timed, every stage
    # bracketed by HIP events
    ctx.profile_stages(None)
    ctx.profile_begin(steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        pipe.step(x, y, z, h)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    prof = ctx.profile_end()
    # the timed steps: events bracket only the dominant stage (its kernel is
    # the roofline line's); a timing event makes the stream drain the work
    # before it, so bracketing every stage would slow the step
    dom = max((k for k, v in prof.items() if v[1]), key=lambda k: prof[k][0] / prof[k][1])
    ctx.profile_stages([dom])
    ctx.profile_begin(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pipe.step(x, y, z, h)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timed = ctx.profile_end()
    prof[dom] = timed[dom]
    prof["_ms_all_stages_bracketed"] = ((t3 - t2) * 1e3 / steps, 0)
    prof["_live"] = (dom, 0)
    st = list_stats(sf, ctx, pipe.nl)
    del pipe, x, y, z, h
    torch.cuda.empty_cache()
    return (t1 - t0) * 1e3 / steps, prof, st


def stage_table(prof, st, n, half, counters):
    """Per stage: event time, the algorithmic rate against its bound, the
    stage's lower-bound time max(bytes / HBM peak, flops / FP32 peak), and
    (where the committed counters cover every kernel of the stage) the HBM
    bytes the counters saw per step as a fraction of the HBM peak."""
    stages = {}
    for name, (ms, calls) in prof.items():
        if calls == 0 or name.startswith("_"):
            continue
        avg = ms / calls
        d = {"ms": avg}
        byts = BYTES_PER_PARTICLE.get(name, 0) * n
        flops = 0.0
        if name == "traverse":
            flops = st["tile_pairs"] * FLOPS_PER_TEST
            byts += 6.0 * st["entries"]  # staging list entries written
        elif name == "pass":
            flops = st["tile_pairs"] * (FLOPS_PER_PAIR_HALF if half else FLOPS_PER_PAIR)
            byts += st["bytes_per_particle"] * n
        elif name == "encode":
            byts = 6.0 * st["entries"] + st["bytes_per_particle"] * n
        if flops:
            tf = flops / (avg * 1e-3) / 1e12
            d.update(bound="alu", achieved=tf, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s", frac=tf / FP32_PEAK_TFLOPS)
        elif name in BYTES_PER_PARTICLE or name == "encode":
            gbs = byts / (avg * 1e-3) / 1e9
            d.update(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=gbs / HBM_PEAK_GBS)
        d["bound_ms"] = max(byts / (HBM_PEAK_GBS * 1e9), flops / (FP32_PEAK_TFLOPS * 1e12)) * 1e3
        ks = STAGE_KERNELS.get(name)
        if ks and all(k in counters for k in ks):
            cb = sum(counters[k][0] * counters[k][1] for k in ks)
            d["counter_bytes"] = cb
            d["counter_frac"] = cb / (avg * 1e-3) / (HBM_PEAK_GBS * 1e9)
        stages[name] = d
    return stages


def extra_config(sf, torch, ctx, args, name):
    """Build + pass throughput of another configuration: the 32,768-particle
    uniform system with one global radius, or the 8,388,608-particle 1/r
    sphere at radii iterated to 100 +- 1 neighbours (from the analytic-density
    seed, untimed), both in the launch configuration of the main run."""
    from paper_2602_19873_amd import workloads
    if name == "uniform_32k":
        s = workloads.make_config("uniform_32k")
        note = "h = r_c for all"
    else:
        s = workloads.evrard_sphere(8388608, workloads.SEED_BASE + 3, target=100, seed_h="analytic")
        dev = torch.device("cuda:0")
        x, y, z, h = (torch.from_numpy(a).to(dev) for a in (s.x, s.y, s.z, s.h))
        keys, perm = sf.sfc_sort(ctx, x, y, z, s.box)
        xs, ys, zs, hs = sf.sfc_gather(ctx, perm, [x, y, z, h])
        res = sf.h_iterate(ctx, keys, xs, ys, zs, hs, target=100, tol=1, max_iters=64)
        if not res.converged:
            raise RuntimeError("sphere did not converge")
        s.x, s.y, s.z, s.h = (t.cpu().numpy() for t in (xs, ys, zs, hs))
        note = "radii iterated to 100 +- 1 (%d rounds from the analytic seed)" % res.iters
        del keys, perm, x, y, z, h, xs, ys, zs, hs, res
        torch.cuda.empty_cache()
    steps = max(5, args.steps // 2)
    ms, prof, st = time_steps(sf, torch, ctx, s, args, steps, args.warmup)
    build = sum(v[0] / v[1] for k, v in prof.items() if v[1] and k != "pass" and not k.startswith("_"))
    pas = prof["pass"][0] / prof["pass"][1] if prof.get("pass", (0, 0))[1] else 0.0
    log("%s: n=%d %.3f ms/step (build %.3f, pass %.3f) %.3f B/p" % (name, s.n, ms, build, pas,
                                                                    st["bytes_per_particle"]))
    return {"n": s.n, "radii": note, "ms_per_step": ms, "mparticles_per_s": s.n / (ms * 1e-3) / 1e6,
            "build_ms": build, "pass_ms": pas, "mparticles_per_s_events": s.n / ((build + pas) * 1e-3) / 1e6,
            "bytes_per_particle": st["bytes_per_particle"], "mean_nj": st["mean_nj"],
            "tile_pairs_per_particle": st["tile_pairs"] / s.n}


def run_step(args, sf, torch, ctx):
    s = make_workload(args.workload)
    n = s.n
    log("workload %s n=%d" % (args.workload, n))
    ms_step, prof, st = time_steps(sf, torch, ctx, s, args, args.steps, args.warmup, args.copy_probe)
    value = n / (ms_step * 1e-3) / 1e6
    log("timed %d steps: %.3f ms/step" % (args.steps, ms_step))
    counters = read_counters(n)
    stages = stage_table(prof, st, n, bool(args.half), counters)
    dom = prof["_live"][0]  # the dominant stage, timed live in the timed steps
    dd = stages[dom]
    hb = "true" if args.half else "false"
    kernel_of = {"traverse": "k_traverse<%d,%s,false>" % (args.cluster_size, hb),
                 "pass": ("k_pass_half<%d,true,false,true,false>" % args.cluster_size if args.half
                          else "k_pass<%d,true,false,true,false>" % args.cluster_size)}
    kern = kernel_of.get(dom, dom)
    traffic = counters[kern][0] if kern in counters else None
    roofline = {"kernel": kern, "bound": dd["bound"], "achieved": dd["achieved"],
                "peak": dd["peak"], "unit": dd["unit"], "frac": dd["frac"], "traffic": traffic,
                "avg_ms": dd["ms"]}
    bound_sum = sum(v["bound_ms"] for v in stages.values())
    additive = {"sum_stage_bound_ms": bound_sum, "measured_ms": ms_step, "frac": bound_sum / ms_step,
                "note": "sum over stages of max(bytes / 8 TB/s, flops / 157.3 TFLOP/s), over the measured step"}

    out = {
        "metric": METRIC, "value": value, "unit": "Mparticles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "cluster_size": args.cluster_size, "super_cluster": 64,
                   "compress": bool(args.compress), "leaf_bucket": args.leaf_bucket, "radii": "r_c*U(0.8,1.2)",
                   "list": "half (each pair once, j > i)" if args.half else "full",
                   "target_neighbours": 200},
        "bytes_per_particle": st["bytes_per_particle"],
        "list": st,
        "stages_ms": {k: v["ms"] for k, v in stages.items()},
        "stages_note": "stage times from %d more steps with every stage bracketed by HIP events (%.3f ms per step "
                       "there); the dominant stage (%s, the roofline kernel's) from the timed steps, where only it "
                       "is bracketed" % (args.steps, prof["_ms_all_stages_bracketed"][0], dom),
        "stages": stages,
        "roofline": roofline,
        "roofline_additive": additive,
    }
    if not args.no_extra:
        out["configs"] = {name: extra_config(sf, torch, ctx, args, name) for name in ("uniform_32k", "evrard_8m")}
        # the learned seed on the 8M sphere (and on its training generator at
        # 8M) against the plain iteration, and the 64-system batch, each with
        # one untimed and one timed run (the other modes' lines time more)
        import copy
        ha = copy.copy(args)
        ha.steps, ha.warmup, ha.mlp, ha.target, ha.n = 1, 1, 1, 100, 0
        hr = run_hiter(ha, sf, torch, ctx)
        out["configs"]["evrard_8m_hiter"] = {k: hr[k] for k in ("metric", "value", "unit", "ms_per_step", "config",
                                                               "systems", "seed_training")}
        ba = copy.copy(args)
        ba.steps, ba.warmup, ba.target = 1, 1, 150
        br = run_batch(ba, sf, torch, ctx)
        out["configs"]["batch_64"] = {k: br[k] for k in ("metric", "value", "unit", "ms_per_step", "config",
                                                        "batched_seeded_graph", "plain_per_system",
                                                        "batched_plain_graph", "seeded_per_system",
                                                        "speedup_vs_plain_per_system", "autotune")}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) on %d particles" % n)
        out["cpu_baseline"] = cpu_baseline(s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
