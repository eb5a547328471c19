"""CPU oracle for the SFC cluster neighbour list and the SPH density pass.

TEST INFRASTRUCTURE ONLY: plain, slow, obviously correct reference code that
the GPU library is checked against. Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the GPU library never does,
and the two share no code.

Every function cites the part of the paper it follows ("GPU-Native Compressed
Neighbor Lists with a Space-Filling-Curve Data Layout"). The heavy loops live
in ``oracle.c`` (built with gcc, ``-ffp-contract=off``); library primitives
(numpy's stable argsort, min/max) serve as single steps.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

KEY_BITS = 21
SC_SIZE = 64   # particles per super-cluster (Sec. II-A)
WAVE = 64      # segment width: the AMD wavefront (Sec. II-C)


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (no GPU code involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build()
        lib = C.CDLL(_LIB)
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        u16p = np.ctypeslib.ndpointer(np.uint16, flags="C_CONTIGUOUS")
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        lib.orc_hilbert3.restype = C.c_uint64
        lib.orc_hilbert3.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_int]
        lib.orc_hilbert_keys.restype = None
        lib.orc_hilbert_keys.argtypes = [C.c_int64, f32p, f32p, f32p, f32p, u64p]
        lib.orc_is_pair.restype = C.c_int
        lib.orc_is_pair.argtypes = [C.c_float] * 8
        lib.orc_max_degree.restype = C.c_int64
        lib.orc_max_degree.argtypes = [C.c_int64, f32p, f32p, f32p, f32p, C.c_int, f32p]
        lib.orc_pairs_csr.restype = None
        lib.orc_pairs_csr.argtypes = [C.c_int64, f32p, f32p, f32p, f32p, C.c_int, i64p, C.c_void_p, f32p]
        lib.orc_cluster_list.restype = C.c_int
        lib.orc_cluster_list.argtypes = [C.c_int64, f32p, f32p, f32p, f32p, C.c_int, C.c_int, C.c_int, C.c_int64,
                                         C.c_void_p, C.c_int64, C.POINTER(C.c_void_p),
                                         C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), f32p]
        lib.orc_free.restype = None
        lib.orc_free.argtypes = [C.c_void_p]
        lib.orc_encode_block_symbols.restype = C.c_int
        lib.orc_encode_block_symbols.argtypes = [u32p, C.c_int, u8p, u8p, C.POINTER(C.c_int), u8p,
                                                 C.POINTER(C.c_int)]
        lib.orc_encode_sc.restype = C.c_int64
        lib.orc_encode_sc.argtypes = [C.c_int64, u32p, u16p, C.c_int, C.c_int, C.c_void_p]
        lib.orc_decode_sc.restype = C.c_int64
        lib.orc_decode_sc.argtypes = [u32p, C.c_int64, C.c_int, C.c_int, u32p, u16p]
        lib.orc_encode_row.restype = C.c_int64
        lib.orc_encode_row.argtypes = [C.c_int64, u32p, C.c_int, C.c_void_p]
        lib.orc_decode_row.restype = C.c_int64
        lib.orc_decode_row.argtypes = [u32p, C.c_int64, C.c_int, u32p]
        lib.orc_kernel_w.restype = C.c_double
        lib.orc_kernel_w.argtypes = [C.c_double, C.c_double]
        lib.orc_density.restype = None
        lib.orc_density.argtypes = [C.c_int64, f32p, f32p, f32p, f32p, C.c_void_p, C.c_int, f64p, i32p, f32p]
        lib.orc_lj.restype = None
        lib.orc_lj.argtypes = [C.c_int64, f32p, f32p, f32p, C.c_void_p, C.c_double, C.c_double, C.c_double,
                               C.c_float, C.c_int, C.c_void_p, C.c_int64, f64p, f64p, f64p, f64p, i32p, f32p]
        lib.orc_num_threads.restype = C.c_int
        lib.orc_num_threads.argtypes = []
        lib.orc_set_num_threads.restype = None
        lib.orc_set_num_threads.argtypes = [C.c_int]
        _lib = lib
        return lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _per(period):
    """Periods as 3 float32 (0 = open axis); None = all open (Sec. II-A:
    periodic boundaries by minimum images, no shift vectors)."""
    if period is None:
        return np.zeros(3, np.float32)
    p = _f32(period).reshape(-1)
    if p.shape[0] != 3 or not np.all(np.isfinite(p)) or np.any(p < 0):
        raise ValueError("period must be 3 finite values >= 0")
    return p


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(k: int) -> None:
    """OpenMP threads of the following oracle calls."""
    _load().orc_set_num_threads(int(k))


# --------------------------------------------------------------------------
# Sec. II-A: Hilbert order, stable sort, clusters
# --------------------------------------------------------------------------

def hilbert3(x: int, y: int, z: int, bits: int = KEY_BITS) -> int:
    """Hilbert index of integer cell (x, y, z) on a 2^bits grid (Skilling)."""
    return int(_load().orc_hilbert3(x, y, z, bits))


def hilbert_keys(x, y, z, box) -> np.ndarray:
    """63-bit keys of positions quantised to 21 bits per axis inside box
    = (xmin, xmax, ymin, ymax, zmin, zmax)."""
    x, y, z = _f32(x), _f32(y), _f32(z)
    out = np.empty(x.shape[0], dtype=np.uint64)
    _load().orc_hilbert_keys(x.shape[0], x, y, z, _f32(box), out)
    return out


def sfc_order(keys) -> np.ndarray:
    """Permutation putting particles in ascending key order, ties kept in
    input order (a stable sort; library primitive)."""
    return np.argsort(np.asarray(keys), kind="stable").astype(np.uint32)


def cluster_bboxes(x, y, z, h, cs: int) -> np.ndarray:
    """Per cluster of cs consecutive particles: (lo.x, lo.y, lo.z, h_max,
    hi.x, hi.y, hi.z, 0) as float32 (exact min / max)."""
    n = len(x)
    nc = (n + cs - 1) // cs
    out = np.zeros((nc, 8), dtype=np.float32)
    for c in range(0, nc):
        s = slice(c * cs, min(n, c * cs + cs))
        out[c, 0], out[c, 1], out[c, 2] = x[s].min(), y[s].min(), z[s].min()
        out[c, 3] = h[s].max()
        out[c, 4], out[c, 5], out[c, 6] = x[s].max(), y[s].max(), z[s].max()
    return out


# --------------------------------------------------------------------------
# Sec. II-A: pair set and cluster-pair list
# --------------------------------------------------------------------------

def is_pair(xi, yi, zi, hi, xj, yj, zj, hj) -> bool:
    return bool(_load().orc_is_pair(xi, yi, zi, hi, xj, yj, zj, hj))


def pairs_csr(x, y, z, h, method: str = "brute", period=None):
    """Pair set P as CSR (offs[n+1], nbr ascending per particle); period: 3
    lengths (0 = open axis) for periodic boundaries."""
    x, y, z, h = _f32(x), _f32(y), _f32(z), _f32(h)
    n = x.shape[0]
    g = 1 if method == "grid" else 0
    per = _per(period)
    offs = np.zeros(n + 1, dtype=np.int64)
    lib = _load()
    lib.orc_pairs_csr(n, x, y, z, h, g, offs, None, per)
    nbr = np.zeros(max(1, int(offs[-1])), dtype=np.int64)
    lib.orc_pairs_csr(n, x, y, z, h, g, offs, nbr.ctypes.data, per)
    return offs, nbr[: offs[-1]]


def max_degree(x, y, z, h, method: str = "grid", period=None) -> int:
    x, y, z, h = _f32(x), _f32(y), _f32(z), _f32(h)
    return int(_load().orc_max_degree(x.shape[0], x, y, z, h, 1 if method == "grid" else 0, _per(period)))


def cluster_list(x, y, z, h, cs: int = 8, method: str = "grid", sc_ids=None, half: bool = False, period=None):
    """Cluster-pair list of Sec. II-A: per selected super-cluster the
    ascending j-cluster indices and their i-cluster bitmasks. half: only
    pairs with j > i count (each pair of P stored once, Sec. II-D's symmetric
    option). period: periodic axes (minimum images; one entry per j-cluster
    whatever image its pairs use, Sec. II-A's list without shift vectors).

    Returns (offs[nsel+1] int64, j uint32, mask uint16)."""
    x, y, z, h = _f32(x), _f32(y), _f32(z), _f32(h)
    n = x.shape[0]
    lib = _load()
    g = 1 if method == "grid" else 0
    md = 1024  # initial neighbour buffer; grows on demand
    if sc_ids is None:
        nsel = (n + SC_SIZE - 1) // SC_SIZE
        ids_ptr = None
        ids = None
    else:
        ids = np.ascontiguousarray(sc_ids, dtype=np.int64)
        nsel = ids.shape[0]
        ids_ptr = ids.ctypes.data
    po, pj, pm = C.c_void_p(), C.c_void_p(), C.c_void_p()
    rc = lib.orc_cluster_list(n, x, y, z, h, cs, int(bool(half)), g, nsel, ids_ptr, md, C.byref(po), C.byref(pj),
                              C.byref(pm), _per(period))
    if rc != 0:
        raise MemoryError("oracle cluster list")
    offs = np.ctypeslib.as_array(C.cast(po, C.POINTER(C.c_int64)), shape=(nsel + 1,)).copy()
    tot = int(offs[-1])
    j = np.ctypeslib.as_array(C.cast(pj, C.POINTER(C.c_uint32)), shape=(max(tot, 1),))[:tot].copy()
    m = np.ctypeslib.as_array(C.cast(pm, C.POINTER(C.c_uint16)), shape=(max(tot, 1),))[:tot].copy()
    for p in (po, pj, pm):
        lib.orc_free(p)
    return offs, j, m


# --------------------------------------------------------------------------
# Sec. II-B / II-C: nibble encoding
# --------------------------------------------------------------------------

def block_symbols(values):
    """Symbols of one block of difference values (Sec. II-B): (bitmask as a
    0/1 list, info nibbles, data nibbles)."""
    v = np.ascontiguousarray(values, dtype=np.uint32)
    cnt = v.shape[0]
    bits = np.zeros(max(cnt, 1), np.uint8)
    info = np.zeros(max(cnt, 1), np.uint8)
    data = np.zeros(max(cnt * 8, 1), np.uint8)
    ni, nd = C.c_int(0), C.c_int(0)
    if _load().orc_encode_block_symbols(v, cnt, bits, info, C.byref(ni), data, C.byref(nd)) != 0:
        raise ValueError("difference value 0 cannot be encoded")
    return list(bits[:cnt]), list(info[: ni.value]), list(data[: nd.value])


def encode_sc(j, mask, cs: int = 8, compress: bool = True) -> np.ndarray:
    """Word stream (uint32) of one super-cluster: masks, then the j indices
    (raw or in nibble segments)."""
    j = np.ascontiguousarray(j, dtype=np.uint32)
    mask = np.ascontiguousarray(mask, dtype=np.uint16)
    lib = _load()
    nw = lib.orc_encode_sc(j.shape[0], j, mask, cs, int(compress), None)
    if nw < 0:
        raise ValueError("list not strictly ascending")
    out = np.zeros(max(int(nw), 1), dtype=np.uint32)
    lib.orc_encode_sc(j.shape[0], j, mask, cs, int(compress), out.ctypes.data)
    return out[: int(nw)]


def decode_sc(words, nj: int, cs: int = 8, compress: bool = True):
    w = np.ascontiguousarray(words, dtype=np.uint32)
    if w.shape[0] == 0:
        w = np.zeros(1, np.uint32)
    j = np.zeros(max(nj, 1), np.uint32)
    m = np.zeros(max(nj, 1), np.uint16)
    used = _load().orc_decode_sc(w, nj, cs, int(compress), j, m)
    if used < 0:
        raise ValueError("malformed stream")
    return j[:nj], m[:nj], int(used)


def encode_row(j, compress: bool = True) -> np.ndarray:
    """Word stream of one 1x1 row (the paper's future-work combination of the
    compression with a full neighbour list, Sec. V): the ascending indices as
    the index stream of a super-cluster list, with no masks."""
    j = np.ascontiguousarray(j, dtype=np.uint32)
    lib = _load()
    nw = lib.orc_encode_row(j.shape[0], j, int(compress), None)
    if nw < 0:
        raise ValueError("row not strictly ascending")
    out = np.zeros(max(int(nw), 1), dtype=np.uint32)
    lib.orc_encode_row(j.shape[0], j, int(compress), out.ctypes.data)
    return out[: int(nw)]


def decode_row(words, nj: int, compress: bool = True):
    w = np.ascontiguousarray(words, dtype=np.uint32)
    if w.shape[0] == 0:
        w = np.zeros(1, np.uint32)
    j = np.zeros(max(nj, 1), np.uint32)
    used = _load().orc_decode_row(w, nj, int(compress), j)
    if used < 0:
        raise ValueError("malformed stream")
    return j[:nj], int(used)


def row_list(x, y, z, h, compress: bool = True, method: str = "grid", period=None):
    """The compressed 1x1 list: per particle its ascending neighbours in P
    (j != i, d2 < max(h_i, h_j)^2), rows laid out in particle order.
    Returns (info (n x 2 uint32: word offset, count), pool uint32)."""
    offs, nbr = pairs_csr(x, y, z, h, method, period=period)
    n = offs.shape[0] - 1
    info = np.zeros((n, 2), dtype=np.uint32)
    parts, pos = [], 0
    for i in range(n):
        a, b = int(offs[i]), int(offs[i + 1])
        words = encode_row(nbr[a:b].astype(np.uint32), compress) if b > a else np.zeros(0, np.uint32)
        info[i] = (pos, b - a)
        parts.append(words)
        pos += words.shape[0]
    pool = np.concatenate(parts) if parts else np.zeros(0, np.uint32)
    return info, pool


def encode_all(offs, j, mask, cs: int = 8, compress: bool = True):
    """Whole list: sc_info (n_sc x 2 uint32: word offset, n_j) and the pool
    (uint32 words), super-clusters laid out in order."""
    nsc = offs.shape[0] - 1
    info = np.zeros((nsc, 2), dtype=np.uint32)
    parts = []
    pos = 0
    for s in range(nsc):
        a, b = int(offs[s]), int(offs[s + 1])
        words = encode_sc(j[a:b], mask[a:b], cs, compress) if b > a else np.zeros(0, np.uint32)
        info[s, 0] = pos
        info[s, 1] = b - a
        parts.append(words)
        pos += words.shape[0]
    pool = np.concatenate(parts) if parts else np.zeros(0, np.uint32)
    return info, pool


# --------------------------------------------------------------------------
# Sec. II-D, Listing 1: SPH density and neighbour counts (FP64)
# --------------------------------------------------------------------------

def kernel_w(r: float, h: float) -> float:
    return float(_load().orc_kernel_w(r, h))


def density(x, y, z, h, m=None, method: str = "grid", period=None):
    """(rho float64, nnb int32): gather density with support h_i and the
    number of j != i inside h_i (decided by the FP32 pair formula, minimum
    images on periodic axes)."""
    x, y, z, h = _f32(x), _f32(y), _f32(z), _f32(h)
    n = x.shape[0]
    rho = np.zeros(max(n, 1), np.float64)
    nnb = np.zeros(max(n, 1), np.int32)
    mm = None if m is None else _f32(m)
    _load().orc_density(n, x, y, z, h, None if mm is None else mm.ctypes.data,
                        1 if method == "grid" else 0, rho, nnb, _per(period))
    return rho[:n], nnb[:n]


# --------------------------------------------------------------------------
# Sec. III, Lennard-Jones benchmark: 12/6 Lennard-Jones + Coulomb forces of
# the pairs inside an interaction cutoff shorter than the list cutoff (FP64)
# --------------------------------------------------------------------------

def lj(x, y, z, q=None, eps: float = 1.0, sigma: float = 1.0, coulomb: float = 0.0, r_cut: float = 1.0,
       method: str = "grid", idx=None, period=None):
    """Pair forces of U(r) = 4 eps ((sigma/r)^12 - (sigma/r)^6) + k q_i q_j / r
    over the pairs j != i with d2 < f32(r_cut^2) (the FP32 pair formula).

    Returns dict(f=(rows, 3) float64 forces on i, e=per-particle energy (half of
    each pair's), scale=sum_j |F_ij| and escale=sum_j |U_ij| / 2 (for rounding
    bounds), nnb=pairs per particle). ``idx`` restricts the rows to those
    particles."""
    x, y, z = _f32(x), _f32(y), _f32(z)
    n = x.shape[0]
    qq = None if q is None else _f32(q)
    ii = None if idx is None else np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    rows = n if ii is None else ii.shape[0]
    f = np.zeros((max(rows, 1), 3), np.float64)
    e = np.zeros(max(rows, 1), np.float64)
    sc = np.zeros(max(rows, 1), np.float64)
    esc = np.zeros(max(rows, 1), np.float64)
    nnb = np.zeros(max(rows, 1), np.int32)
    _load().orc_lj(n, x, y, z, None if qq is None else qq.ctypes.data, float(eps), float(sigma), float(coulomb),
                   float(r_cut), 1 if method == "grid" else 0, None if ii is None else ii.ctypes.data, rows,
                   f.reshape(-1), e, sc, esc, nnb, _per(period))
    return dict(f=f[:rows], e=e[:rows], scale=sc[:rows], escale=esc[:rows], nnb=nnb[:rows])


# --------------------------------------------------------------------------
# The whole path on one system
# --------------------------------------------------------------------------

def pipeline(x, y, z, h, box, m=None, cs: int = 8, compress: bool = True, method: str = "grid",
             half: bool = False, period=None):
    """Hilbert keys -> stable order -> SFC-ordered arrays -> cluster list ->
    encoding -> density, all in SFC order. Returns a dict."""
    keys = hilbert_keys(x, y, z, box)
    perm = sfc_order(keys)
    xs, ys, zs, hs = (np.asarray(a)[perm] for a in (x, y, z, h))
    ms = None if m is None else np.asarray(m)[perm]
    offs, jj, mm = cluster_list(xs, ys, zs, hs, cs, method, half=half, period=period)
    info, pool = encode_all(offs, jj, mm, cs, compress)
    rho, nnb = density(xs, ys, zs, hs, ms, method, period=period)
    return dict(keys=keys, perm=perm, sorted_keys=keys[perm], x=xs, y=ys, z=zs, h=hs, m=ms,
                offs=offs, j=jj, mask=mm, sc_info=info, pool=pool, rho=rho, nnb=nnb)


# --------------------------------------------------------------------------
# Smoothing-length iteration (not from the paper: the rule this project uses
# to drive each particle to a target own-radius neighbour count; the paper
# rebuilds its list every step with per-particle radii, Sec. IV)
# --------------------------------------------------------------------------

def h_step(h, cnt, lo, hi, target: int, tol: int):
    """One round of the rule for every particle, given its radius h, its
    own-radius count cnt and its bracket [lo, hi] (lo = 0 and hi = inf while
    open). A particle with |cnt - target| <= tol keeps everything. Otherwise
    its bracket narrows first (lo = max(lo, h) when too few, hi = min(hi, h)
    when too many); the proposal is 2h for cnt = 0, else h (target/cnt)^(1/3)
    clamped to [h/2, 2h]; a proposal not strictly inside (lo, hi) becomes the
    midpoint, or 2 lo while hi is open, or hi/2 while lo is open. FP64.
    Returns (h_new float64, lo, hi, moved)."""
    hc = np.asarray(h, dtype=np.float64)
    cnt = np.asarray(cnt, dtype=np.int64)
    lo = np.array(lo, dtype=np.float64, copy=True)
    hi = np.array(hi, dtype=np.float64, copy=True)
    dev = cnt - target
    move = np.abs(dev) > tol
    few = move & (dev < 0)
    many = move & (dev > 0)
    lo[few] = np.maximum(lo[few], hc[few])
    hi[many] = np.minimum(hi[many], hc[many])
    with np.errstate(divide="ignore"):
        hn = np.where(cnt == 0, 2.0 * hc, hc * np.cbrt(target / np.maximum(cnt, 1)))
    hn = np.where(cnt == 0, hn, np.clip(hn, 0.5 * hc, 2.0 * hc))
    out = ~((hn > lo) & (hn < hi))
    mid = np.where(np.isinf(hi), 2.0 * lo, np.where(lo == 0.0, 0.5 * hi, 0.5 * (lo + hi)))
    hn = np.where(out, mid, hn)
    return np.where(move, hn, hc), lo, hi, move


def h_iterate(x, y, z, h0, target: int, tol: int = 1, max_iters: int = 64, method: str = "grid"):
    """Plain reference of the rule: h_step() on the counts of density() each
    round until every particle is within target +- tol; h is stored in FP32
    between rounds. Returns (h, rounds, unconverged)."""
    h = np.ascontiguousarray(h0, dtype=np.float32).copy()
    n = h.shape[0]
    lo = np.zeros(n)
    hi = np.full(n, np.inf)
    for it in range(max_iters):
        _, cnt = density(x, y, z, h, None, method)
        hn, lo, hi, move = h_step(h, cnt, lo, hi, target, tol)
        if not move.any():
            return h, it + 1, 0
        h = hn.astype(np.float32)
    _, cnt = density(x, y, z, h, None, method)
    return h, max_iters, int((np.abs(cnt.astype(np.int64) - target) > tol).sum())


# --------------------------------------------------------------------------
# Learned h-seed (not from the paper): MLP 8 -> 64 -> 64 -> 1 with ReLU whose
# output plus the cube-root rule's step (-feature0 / 3) predicts
# d = log(h_converged / h_prev); MSE loss; Adam.
# Parameter vector layout (4801 floats): W1[64][8], b1[64], W2[64][64], b2[64],
# w3[64], b3.
# --------------------------------------------------------------------------

MLP_SIZES = (("W1", (64, 8)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("w3", (64,)), ("b3", (1,)))
MLP_NPARAM = 4801


def mlp_unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shp in MLP_SIZES:
        k = int(np.prod(shp))
        out[name] = p[o:o + k].reshape(shp)
        o += k
    return out


def mlp_pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in MLP_SIZES])


def bf16(a):
    """Round to bfloat16 (round to nearest, ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def mlp_forward(p, feat, quant=False):
    """feat: (B, 8). With quant, weights, inputs and hidden activations are
    rounded to bfloat16 where the GPU kernels feed them to the matrix cores;
    sums are exact (FP64). Returns (y, cache)."""
    P = mlp_unpack(p)
    q = bf16 if quant else (lambda a: np.asarray(a, dtype=np.float64))
    x = q(feat)
    W1, W2, w3 = q(P["W1"]), q(P["W2"]), q(P["w3"])
    z1 = x @ W1.T + P["b1"]
    h1 = q(np.maximum(z1, 0.0))
    z2 = h1 @ W2.T + P["b2"]
    h2 = q(np.maximum(z2, 0.0))
    # the network learns a residual on the cube-root rule's step
    # log((target / (n+1))^(1/3)) = -feature0 / 3
    y = h2 @ w3 + P["b3"][0] - x[:, 0] / 3.0
    return y, dict(x=x, W1=W1, W2=W2, w3=w3, z1=z1, h1=h1, z2=z2, h2=h2)


def mlp_loss_grad(p, feat, target, quant=False):
    """Mean squared error and its gradient (flat, same layout as p). With
    quant, the back-propagated errors are rounded to bfloat16 before they
    enter matrix products, as in the GPU kernels (bias gradients use the
    unrounded errors)."""
    q = bf16 if quant else (lambda a: np.asarray(a, dtype=np.float64))
    y, c = mlp_forward(p, feat, quant)
    B = y.shape[0]
    r = y - np.asarray(target, dtype=np.float64)
    loss = float(np.mean(r * r))
    dy = 2.0 * r / B
    g = {}
    g["w3"] = c["h2"].T @ dy
    g["b3"] = np.array([dy.sum()])
    d2 = np.outer(dy, c["w3"]) * (c["z2"] > 0)
    g["b2"] = d2.sum(axis=0)
    d2q = q(d2)
    g["W2"] = d2q.T @ c["h1"]
    d1 = (d2q @ c["W2"]) * (c["z1"] > 0)
    g["b1"] = d1.sum(axis=0)
    g["W1"] = q(d1).T @ c["x"]
    return loss, mlp_pack(g)


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015), bias-corrected, step t >= 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def hseed_features(keys_sorted, h, nnb, bbox, edge0: float, target: int, level=None):
    """Features of the learned seed for SFC-ordered particles (float64, before
    rounding to bf16): log((n+1)/T); log(max(cluster box diagonal / h, 1e-3));
    the same for the 64-particle super-cluster box; log((1 + occupancy)/T) of
    the particle's Hilbert-key cell at levels L0-1, L0, L0+1 with
    L0 = clamp(round(log2(edge0 / h)), 2, 20); log2(edge0 / h) - L0;
    log(T / 100). With nnb None (no count yet: the seed applied before the
    first round) the first feature is 0. ``level`` (optional, one integer per
    particle) replaces L0, for checks where FP32 and FP64 round log2(edge0 / h)
    to different levels."""
    keys = np.asarray(keys_sorted, dtype=np.uint64)
    h = np.asarray(h, dtype=np.float64)
    n = h.shape[0]
    lt = math.log(target)
    f = np.zeros((n, 8))
    if nnb is not None:
        f[:, 0] = np.log(np.asarray(nnb, dtype=np.float64) + 1.0) - lt
    bb = np.asarray(bbox, dtype=np.float64).reshape(-1, 8)
    c = np.arange(n) // 8
    diag = np.sqrt(((bb[:, 4:7] - bb[:, 0:3]) ** 2).sum(axis=1))
    f[:, 1] = np.log(np.maximum(diag[c] / h, 1e-3))
    nsc = (bb.shape[0] + 7) // 8
    slo = np.array([bb[8 * k:8 * k + 8, 0:3].min(axis=0) for k in range(nsc)])
    shi = np.array([bb[8 * k:8 * k + 8, 4:7].max(axis=0) for k in range(nsc)])
    sdiag = np.sqrt(((shi - slo) ** 2).sum(axis=1))
    f[:, 2] = np.log(np.maximum(sdiag[c // 8] / h, 1e-3))
    lev = np.log2(edge0 / h)
    L0 = np.clip(np.rint(lev), 2, 20).astype(np.int64)
    if level is not None:
        L0 = np.asarray(level, dtype=np.int64)
    for d in (-1, 0, 1):
        L = L0 + d
        shift = (3 * (21 - L)).astype(np.uint64)
        pre = keys >> shift
        lo = np.searchsorted(keys, pre << shift, side="left")
        hi = np.searchsorted(keys, (pre + np.uint64(1)) << shift, side="left")
        f[:, 4 + d] = np.log(1.0 + (hi - lo)) - lt
    f[:, 6] = lev - L0
    f[:, 7] = lt - math.log(100.0)
    return f
