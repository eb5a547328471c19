"""Compressed SFC cluster neighbour lists on MI355X (gfx950).

Python binding of libsfcnl.so. Functions carry the names of the C ABI and only
marshal arguments: every step runs in the library's HIP kernels. PyTorch
provides device memory and the stream.

Method: "GPU-Native Compressed Neighbor Lists with a Space-Filling-Curve Data
Layout" -- Hilbert order (Sec. II-A), 8-particle clusters and 64-particle
super-clusters (Sec. II-A), octree traversal with per-particle radii
(Sec. II-A), nibble compression (Sec. II-B, II-C) and the neighbour pass
(Sec. II-A, II-D).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib

__all__ = ["Context", "NeighbourList", "SfcnlError", "sfc_sort", "sfc_sort_noalloc", "sfc_gather", "sfc_gather_workspace", "build_clusters",
           "build_nlist", "nlist_pass", "nlist_decode", "h_iterate", "HIterResult", "Pipeline", "SC_SIZE",
           "CLUSTER_SIZE", "hseed_features", "mlp_init", "mlp_infer", "mlp_grad", "mlp_adam", "mlp_train",
           "MLP_NPARAM", "Batch", "batch_create", "batch_sort", "batch_gather", "batch_build_clusters",
           "batch_build_nlist", "batch_pass", "batch_h_iterate", "BatchIterResult"]

SC_SIZE = 64
CLUSTER_SIZE = 8
SEED_AFTER_FIRST = _lib.SEED_AFTER_FIRST
SEED_BEFORE_FIRST = _lib.SEED_BEFORE_FIRST


class SfcnlError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("sfcnl error %d: %s" % (code, msg))
        self.code = code


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_f32(t, n, name):
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError("%s must be a contiguous float32 device tensor of %d elements" % (name, n))


class Context:
    """A library context bound to one device and (by default) torch's current stream."""

    def __init__(self, device: int | None = None, stream: torch.cuda.Stream | None = None):
        self.lib = _lib.load()
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = self.lib.sfcnl_create(C.byref(h), self.device, C.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise SfcnlError(rc, "sfcnl_create failed")
        self.handle = h

    def check(self, rc):
        if rc != 0:
            raise SfcnlError(rc, self.lib.sfcnl_last_error(self.handle).decode())

    def set_pass_waves(self, waves: int):
        """Wavefronts per workgroup of the density passes (1, 2 or 4)."""
        self.check(self.lib.sfcnl_set_pass_waves(self.handle, int(waves)))
        self.pass_waves = int(waves)

    def sync(self):
        self.check(self.lib.sfcnl_sync(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.sfcnl_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile_begin(self, slots: int):
        """Start per-stage event timing (see sfcnl_profile_begin)."""
        self.check(self.lib.sfcnl_profile_begin(self.handle, slots))

    def profile_stages(self, stages=None):
        """Record stage events only for the named stages (None: all)."""
        mask = (1 << _lib.NSTAGE) - 1 if stages is None else sum(1 << _lib.STAGES.index(s) for s in stages)
        self.check(self.lib.sfcnl_profile_stages(self.handle, mask))

    def profile_end(self):
        """Stop stage timing: {stage: (total ms, calls)}."""
        ms = (C.c_double * _lib.NSTAGE)()
        calls = (C.c_int64 * _lib.NSTAGE)()
        self.check(self.lib.sfcnl_profile_end(self.handle, ms, calls))
        return {name: (ms[i], calls[i]) for i, name in enumerate(_lib.STAGES)}

    def empty(self, shape, dtype):
        return torch.empty(shape, dtype=dtype, device="cuda:%d" % self.device)


def sfc_sort_workspace(n: int) -> int:
    b = C.c_size_t()
    if _lib.load().sfc_sort_workspace(n, C.byref(b)) != 0:
        raise SfcnlError(_lib.E_ARG, "sfc_sort_workspace")
    return b.value


def sfc_sort(ctx: Context, x, y, z, box, keys=None, perm=None, ws=None):
    """Hilbert keys and stable SFC order. Returns (sorted keys u64 as int64, perm int32)."""
    n = x.numel()
    for t, nm in ((x, "x"), (y, "y"), (z, "z")):
        _check_f32(t, n, nm)
    keys = ctx.empty(n, torch.int64) if keys is None else keys
    perm = ctx.empty(n, torch.int32) if perm is None else perm
    need = sfc_sort_workspace(n)
    ws = ctx.empty(max(need, 1), torch.uint8) if ws is None or ws.numel() < need else ws
    hb = (C.c_float * 6)(*[float(v) for v in box])
    ctx.check(ctx.lib.sfc_sort(ctx.handle, n, _ptr(x), _ptr(y), _ptr(z), hb, _ptr(keys), _ptr(perm), _ptr(ws),
                               ws.numel()))
    return keys, perm


def sfc_sort_noalloc(ctx: Context, x, y, z, box, keys=None, perm=None):
    """sfc_sort with the library's fixed device scratch instead of a workspace
    (n <= SORT_NOALLOC_MAX_N; no device allocation inside the call)."""
    n = x.numel()
    for t, nm in ((x, "x"), (y, "y"), (z, "z")):
        _check_f32(t, n, nm)
    keys = ctx.empty(n, torch.int64) if keys is None else keys
    perm = ctx.empty(n, torch.int32) if perm is None else perm
    hb = (C.c_float * 6)(*[float(v) for v in box])
    ctx.check(ctx.lib.sfc_sort_noalloc(ctx.handle, n, _ptr(x), _ptr(y), _ptr(z), hb, _ptr(keys), _ptr(perm)))
    return keys, perm


SORT_NOALLOC_MAX_N = _lib.SORT_NOALLOC_MAX_N


def sfc_gather_workspace(n: int) -> int:
    """Bytes of workspace sfc_gather needs to stage its reads (16 n + 256)."""
    b = C.c_size_t()
    if _lib.load().sfc_gather_workspace(int(n), C.byref(b)) != 0:
        raise SfcnlError(_lib.E_ARG, "sfc_gather_workspace")
    return b.value


def sfc_gather(ctx: Context, perm, fields, outs=None, ws=None):
    """out[f][k] = fields[f][perm[k]]. With ws (a uint8 tensor of at least
    sfc_gather_workspace(n) bytes) the fields are staged four at a time into
    16-byte records, one random read per particle (sfc_gather_ws)."""
    n = perm.numel()
    nf = len(fields)
    outs = [torch.empty_like(f) for f in fields] if outs is None else outs
    for f in list(fields) + list(outs):
        _check_f32(f, n, "field")
    ins = (C.c_void_p * nf)(*[f.data_ptr() for f in fields])
    ous = (C.c_void_p * nf)(*[o.data_ptr() for o in outs])
    if ws is None:
        ctx.check(ctx.lib.sfc_gather(ctx.handle, n, _ptr(perm), nf, ins, ous))
    else:
        ctx.check(ctx.lib.sfc_gather_ws(ctx.handle, n, _ptr(perm), nf, ins, ous, _ptr(ws), ws.numel()))
    return outs


def build_clusters(ctx: Context, x, y, z, h, cluster_size: int = CLUSTER_SIZE, bbox=None):
    """Per-cluster boxes (n_clusters x 8 float32: lo xyz, max h, hi xyz, 0)."""
    n = x.numel()
    nc = (n + cluster_size - 1) // cluster_size
    bbox = ctx.empty((max(nc, 1), 8), torch.float32) if bbox is None else bbox
    if bbox.numel() < 8 * nc:
        raise ValueError("bbox holds %d boxes, %d clusters need them" % (bbox.numel() // 8, nc))
    ctx.check(ctx.lib.build_clusters(ctx.handle, n, _ptr(x), _ptr(y), _ptr(z), _ptr(h), cluster_size, _ptr(bbox)))
    return bbox


@dataclass
class NeighbourList:
    n: int
    cluster_size: int
    compress: bool
    sc_info: torch.Tensor     # (n_sc, 2) int32 view of u32 {word offset, n_j}
    pool: torch.Tensor        # int32 view of u32 words
    used_bytes: int
    max_nj: int
    half: bool = False        # only pairs with j > i (each pair once)
    period: tuple = (0.0, 0.0, 0.0)  # periodic axes (0 = open), as built
    pending: bool = False     # built by build_nlist_async: sizes unknown until build_nlist_finish

    @property
    def n_sc(self) -> int:
        return (self.n + SC_SIZE - 1) // SC_SIZE

    def bytes_per_particle(self) -> float:
        return (self.used_bytes + 8 * self.n_sc) / max(self.n, 1)


def _period(period):
    """Periods as a tuple of 3 floats (0 = open axis); None = all open."""
    if period is None:
        return (0.0, 0.0, 0.0)
    p = tuple(float(v) for v in period)
    if len(p) != 3:
        raise ValueError("period needs 3 values (0 = open axis)")
    return p


def _period_arg(period):
    """Host pointer argument for the passes: NULL when every axis is open."""
    p = _period(period)
    return None if not any(p) else (C.c_float * 3)(*p)


def _opts(cluster_size, compress, leaf_bucket, max_j_per_sc, half=False, period=None):
    return _lib.NlistOpts(cluster_size, int(bool(compress)), leaf_bucket, max_j_per_sc, int(bool(half)),
                          (C.c_float * 3)(*_period(period)))


def build_nlist_workspace(n, cluster_size=CLUSTER_SIZE, compress=True, leaf_bucket=128, max_j_per_sc=256,
                          half=False) -> int:
    b = C.c_size_t()
    o = _opts(cluster_size, compress, leaf_bucket, max_j_per_sc, half)
    if _lib.load().build_nlist_workspace(n, C.byref(o), C.byref(b)) != 0:
        raise SfcnlError(_lib.E_ARG, "build_nlist_workspace")
    return b.value


def build_nlist(ctx: Context, keys, x, y, z, h, bbox, compress: bool = True, leaf_bucket: int = 128,
                max_j_per_sc: int = 256, cluster_size: int = CLUSTER_SIZE, pool=None, ws=None, sc_info=None,
                grow: bool = True, half: bool = False, period=None):
    """Builds the compressed cluster-pair list (half: each pair once, j > i;
    period: 3 lengths, 0 = open axis, for periodic boundaries by minimum
    images). Grows the staging list and the pool and retries when the library
    reports they are too small (unless grow=False, which raises)."""
    n = x.numel()
    nsc = (n + SC_SIZE - 1) // SC_SIZE
    sc_info = ctx.empty((max(nsc, 1), 2), torch.int32) if sc_info is None else sc_info
    if pool is None:
        pool = ctx.empty(max(1024, 5 * n), torch.int32)
    while True:
        o = _opts(cluster_size, compress, leaf_bucket, max_j_per_sc, half, period)
        need = build_nlist_workspace(n, cluster_size, compress, leaf_bucket, max_j_per_sc, half)
        if ws is None or ws.numel() < need:
            ws = ctx.empty(max(need, 1), torch.uint8)
        used = C.c_size_t()
        maxnj = C.c_int64()
        rc = ctx.lib.build_nlist(ctx.handle, n, _ptr(keys), _ptr(x), _ptr(y), _ptr(z), _ptr(h), _ptr(bbox),
                                 C.byref(o), _ptr(ws), ws.numel(), _ptr(sc_info), _ptr(pool), pool.numel() * 4,
                                 C.byref(used), C.byref(maxnj))
        if rc == _lib.E_CAPACITY and grow:
            grown = False
            if maxnj.value > max_j_per_sc:
                max_j_per_sc = int(maxnj.value)
                grown = True
            if used.value > pool.numel() * 4:
                pool = ctx.empty(used.value // 4 + 1024, torch.int32)
                grown = True
            if not grown:  # the reported sizes already held: retrying would not change anything
                ctx.check(rc)
            continue
        ctx.check(rc)
        nl = NeighbourList(n, cluster_size, bool(compress), sc_info[:nsc], pool, used.value, maxnj.value,
                           bool(half), _period(period))
        nl.ws = ws
        nl.max_j_per_sc = max_j_per_sc
        return nl


def build_nlist_async(ctx: Context, keys, x, y, z, h, bbox, pool, ws, sc_info, compress: bool = True,
                      leaf_bucket: int = 128, max_j_per_sc: int = 256, cluster_size: int = CLUSTER_SIZE,
                      half: bool = False, period=None):
    """Enqueues the list build without waiting (build_nlist_async). The list
    can be passed at once; build_nlist_finish then reports its sizes and
    errors. Buffers are the caller's (no growth here)."""
    n = x.numel()
    nsc = (n + SC_SIZE - 1) // SC_SIZE
    o = _opts(cluster_size, compress, leaf_bucket, max_j_per_sc, half, period)
    ctx.check(ctx.lib.build_nlist_async(ctx.handle, n, _ptr(keys), _ptr(x), _ptr(y), _ptr(z), _ptr(h), _ptr(bbox),
                                        C.byref(o), _ptr(ws), ws.numel(), _ptr(sc_info), _ptr(pool),
                                        pool.numel() * 4))
    nl = NeighbourList(n, cluster_size, bool(compress), sc_info[:nsc], pool, -1, -1, bool(half), _period(period),
                       pending=True)
    nl.ws = ws
    nl.max_j_per_sc = max_j_per_sc
    return nl


def build_nlist_finish(ctx: Context, nl: NeighbourList) -> bool:
    """Waits for the pending build's status (build_nlist_result) and fills in
    its sizes. True when the list is complete; False when the pool or the
    staging list was too small (nl.used_bytes / nl.max_nj then give the sizes
    needed, and the build and any pass over it must be redone); raises on
    every other error."""
    used = C.c_size_t()
    maxnj = C.c_int64()
    rc = ctx.lib.build_nlist_result(ctx.handle, C.byref(used), C.byref(maxnj))
    nl.used_bytes, nl.max_nj, nl.pending = used.value, maxnj.value, False
    if rc == _lib.E_CAPACITY:
        return False
    ctx.check(rc)
    return True


def nlist_pass(ctx: Context, nl: NeighbourList, x, y, z, h, m=None, rho=None, nnb=None, want_counts=True):
    """SPH density (and neighbour counts) from the compressed list."""
    n = nl.n
    rho = ctx.empty(n, torch.float32) if rho is None else rho
    if want_counts and nnb is None:
        nnb = ctx.empty(n, torch.int32)
    ctx.check(ctx.lib.nlist_pass(ctx.handle, n, nl.cluster_size, int(nl.compress), int(nl.half), _ptr(nl.sc_info),
                                 _ptr(nl.pool), _ptr(x), _ptr(y), _ptr(z), _ptr(h), _ptr(m), _ptr(rho),
                                 _ptr(nnb) if want_counts else None, _period_arg(nl.period)))
    return rho, nnb


def nlist_pass_lj(ctx: Context, nl: NeighbourList, x, y, z, q=None, eps: float = 1.0, sigma: float = 1.0,
                  coulomb: float = 0.0, r_cut: float = 1.0, energy: bool = False, f=None, e=None):
    """Lennard-Jones 12/6 + Coulomb forces over the listed pairs inside r_cut
    (the list built at a radius >= r_cut). Returns (f (3, n) float32 rows fx,
    fy, fz; e per-particle energy or None)."""
    n = nl.n
    for t, nm in ((x, "x"), (y, "y"), (z, "z")) + (((q, "q"),) if q is not None else ()):
        _check_f32(t, n, nm)
    f = ctx.empty((3, max(n, 1)), torch.float32) if f is None else f
    if f.dtype != torch.float32 or not f.is_contiguous() or f.dim() != 2 or f.shape[0] != 3 or f.shape[1] < n:
        raise ValueError("f must be a contiguous float32 (3, >= n) device tensor")
    if energy and e is None:
        e = ctx.empty(max(n, 1), torch.float32)
    par = _lib.LjParams(float(eps), float(sigma), float(coulomb), float(r_cut))
    ctx.check(ctx.lib.nlist_pass_lj(ctx.handle, n, nl.cluster_size, int(nl.compress), int(nl.half),
                                    _ptr(nl.sc_info), _ptr(nl.pool), _ptr(x), _ptr(y), _ptr(z), _ptr(q),
                                    C.byref(par), _ptr(f[0]), _ptr(f[1]), _ptr(f[2]),
                                    _ptr(e) if energy else None, _period_arg(nl.period)))
    return f[:, :n], (e[:n] if energy else None)


@dataclass
class RowList:
    """Compressed 1x1 list (build_rows): per particle its neighbours in order."""
    n: int
    compress: bool
    row_info: torch.Tensor   # (n, 2) int32 view of u32 {word offset, count}
    pool: torch.Tensor       # int32 view of u32 words
    used_bytes: int
    period: tuple = (0.0, 0.0, 0.0)

    def bytes_per_particle(self) -> float:
        return (self.used_bytes + 8 * self.n) / max(self.n, 1)


def build_rows_workspace(n: int) -> int:
    b = C.c_size_t()
    if _lib.load().build_rows_workspace(n, C.byref(b)) != 0:
        raise SfcnlError(_lib.E_ARG, "build_rows_workspace")
    return b.value


def build_rows(ctx: Context, nl: NeighbourList, x, y, z, h, compress: bool = True, pool=None, ws=None,
               row_info=None, grow: bool = True) -> RowList:
    """The compressed 1x1 list from a full cluster list `nl` of the same
    SFC-ordered positions and radii. Grows the pool and retries when it is
    too small (unless grow=False, which raises)."""
    if nl.half:
        raise ValueError("build_rows needs a full cluster list (half=False)")
    n = nl.n
    for t, nm in ((x, "x"), (y, "y"), (z, "z"), (h, "h")):
        _check_f32(t, n, nm)
    need = build_rows_workspace(n)
    if ws is None or ws.numel() < need:
        ws = ctx.empty(max(need, 1), torch.uint8)
    if row_info is None:
        row_info = ctx.empty((max(n, 1), 2), torch.int32)
    if pool is None:
        pool = ctx.empty(max(1024, (40 if compress else 320) * n), torch.int32)
    while True:
        used = C.c_size_t()
        rc = ctx.lib.build_rows(ctx.handle, n, nl.cluster_size, int(nl.compress), _ptr(nl.sc_info), _ptr(nl.pool),
                                _ptr(x), _ptr(y), _ptr(z), _ptr(h), int(bool(compress)), _period_arg(nl.period),
                                _ptr(ws), ws.numel(), _ptr(row_info), _ptr(pool), pool.numel() * 4, C.byref(used))
        if rc == _lib.E_CAPACITY and grow:
            if used.value <= pool.numel() * 4:  # the reported size already held: retrying would not change anything
                ctx.check(rc)
            pool = ctx.empty(used.value // 4 + 1024, torch.int32)
            continue
        ctx.check(rc)
        rl = RowList(n, bool(compress), row_info[:n], pool, used.value, nl.period)
        rl.ws = ws
        return rl


def rows_pass(ctx: Context, rl: RowList, x, y, z, h, m=None, rho=None, nnb=None, want_counts: bool = True):
    """SPH density (and neighbour counts) from the compressed 1x1 list."""
    n = rl.n
    rho = ctx.empty(max(n, 1), torch.float32) if rho is None else rho
    if want_counts and nnb is None:
        nnb = ctx.empty(max(n, 1), torch.int32)
    ctx.check(ctx.lib.rows_pass(ctx.handle, n, int(rl.compress), _ptr(rl.row_info), _ptr(rl.pool), _ptr(x), _ptr(y),
                                _ptr(z), _ptr(h), _ptr(m), _ptr(rho), _ptr(nnb) if want_counts else None,
                                _period_arg(rl.period)))
    return rho[:n], (nnb[:n] if want_counts else None)


def nlist_decode(ctx: Context, nl: NeighbourList):
    """Decodes the list on the device: (offsets int64 host, j uint32 numpy, mask uint16 numpy)."""
    import numpy as np
    info = nl.sc_info.cpu().numpy().view(np.uint32)
    nj = info[:, 1].astype(np.int64)
    offs = np.zeros(nl.n_sc + 1, dtype=np.int64)
    np.cumsum(nj, out=offs[1:])
    total = int(offs[-1])
    d_offs = torch.from_numpy(offs[:-1].astype(np.int32)).to(nl.sc_info.device)
    j = ctx.empty(max(total, 1), torch.int32)
    m = ctx.empty(max(total, 1), torch.int16)
    ctx.check(ctx.lib.nlist_decode(ctx.handle, nl.n, nl.cluster_size, int(nl.compress), _ptr(nl.sc_info),
                                   _ptr(nl.pool), _ptr(d_offs), _ptr(j), _ptr(m)))
    torch.cuda.synchronize(nl.sc_info.device)
    return offs, j[:total].cpu().numpy().view(np.uint32), m[:total].cpu().numpy().view(np.uint16)


@dataclass
class HIterResult:
    iters: int            # rounds run (over all resumed calls)
    unconverged: int      # particles outside target +- tol after the last round
    converged: bool
    nl: NeighbourList     # list at the final radii (valid when converged)
    rho: torch.Tensor
    nnb: torch.Tensor
    moved: int = 0        # sum over rounds of the particles that moved

    def mean_rounds(self) -> float:
        return self.moved / max(self.nl.n, 1) + 1.0


def h_iterate(ctx: Context, keys, x, y, z, h, target: int = 100, tol: int = 1, max_iters: int = 64, m=None,
              compress: bool = True, leaf_bucket: int = 128, max_j_per_sc: int = 256, bracket=None, bbox=None,
              ws=None, pool=None, sc_info=None, rho=None, nnb=None, raise_noconv: bool = False,
              resume: bool = False, mlp_params=None, box_edge: float = 0.0, seed_scratch=None,
              seed_mode: int = _lib.SEED_AFTER_FIRST, cluster_size: int = CLUSTER_SIZE, half: bool = False,
              period=None, recount: int = 0):
    """Iterates the SFC-ordered radii h (updated in place) to target +- tol
    own-radius neighbours (sfcnl_h_iterate). With mlp_params the first round's
    update comes from the learned seed. Grows list buffers and resumes when
    the library reports them too small."""
    n = x.numel()
    nsc = (n + SC_SIZE - 1) // SC_SIZE
    nc = (n + cluster_size - 1) // cluster_size
    e = ctx.empty
    bracket = e(max(2 * n, 2), torch.float32) if bracket is None else bracket
    bbox = e((max(nc, 1), 8), torch.float32) if bbox is None else bbox
    if bbox.numel() < 8 * nc:
        raise ValueError("bbox holds %d boxes, %d clusters need them" % (bbox.numel() // 8, nc))
    sc_info = e((max(nsc, 1), 2), torch.int32) if sc_info is None else sc_info
    pool = e(max(1024, 6 * n), torch.int32) if pool is None else pool
    rho = e(max(n, 1), torch.float32) if rho is None else rho
    nnb = e(max(n, 1), torch.int32) if nnb is None else nnb
    hs = None
    if mlp_params is not None:
        if not box_edge > 0:
            raise ValueError("box_edge must be given with mlp_params")
        if seed_scratch is None:
            seed_scratch = (e((max(n, 1), _lib.HSEED_NFEAT), torch.int16), e(max(n, 1), torch.float32))
        hs = _lib.HSeed(mlp_params.data_ptr(), seed_scratch[0].data_ptr(), seed_scratch[1].data_ptr(), box_edge,
                        seed_mode)
    total, moved, resume = 0, 0, int(bool(resume))
    while True:
        if total >= max_iters:
            nl = NeighbourList(n, cluster_size, bool(compress), sc_info[:nsc], pool, 0, 0, bool(half),
                               _period(period))
            return HIterResult(total, n, False, nl, rho, nnb, moved)
        need = build_nlist_workspace(n, cluster_size, compress, leaf_bucket, max_j_per_sc, half)
        if ws is None or ws.numel() < need:
            ws = e(max(need, 1), torch.uint8)
        no = _opts(cluster_size, compress, leaf_bucket, max_j_per_sc, half, period)
        io = _lib.HiterOpts(target, tol, max_iters - total, resume, int(recount))
        st = _lib.HiterStats()
        seed_arg = C.byref(hs) if (hs is not None and total == 0) else None
        rc = ctx.lib.sfcnl_h_iterate(ctx.handle, n, _ptr(keys), _ptr(x), _ptr(y), _ptr(z), _ptr(h), _ptr(bracket),
                                     _ptr(m), C.byref(no), C.byref(io), _ptr(bbox), _ptr(ws), ws.numel(),
                                     _ptr(sc_info), _ptr(pool), pool.numel() * 4, _ptr(rho), _ptr(nnb), seed_arg,
                                     C.byref(st))
        total += st.iters
        moved += st.moved
        if rc == _lib.E_CAPACITY:
            if st.max_nj > max_j_per_sc:
                max_j_per_sc = int(st.max_nj)
            if st.used_bytes > pool.numel() * 4:
                pool = e(st.used_bytes // 4 + 1024, torch.int32)
            if st.unconverged == 0 and st.iters > 0:
                # converged, only the closing list of the final radii did not
                # fit: build it with room (radii, rho and nnb are final)
                build_clusters(ctx, x, y, z, h, cluster_size, bbox)
                nl = build_nlist(ctx, keys, x, y, z, h, bbox, compress, leaf_bucket, max_j_per_sc, cluster_size,
                                 pool=pool, ws=ws, sc_info=sc_info, half=half, period=period)
                return HIterResult(total, 0, True, nl, rho, nnb, moved)
            # the round that overflowed did not update h (only completed
            # rounds are counted): run it again with room
            resume = 1
            continue
        nl = NeighbourList(n, cluster_size, bool(compress), sc_info[:nsc], pool, st.used_bytes, st.max_nj,
                           bool(half), _period(period))
        nl.ws, nl.max_j_per_sc = ws, max_j_per_sc
        if rc == _lib.E_NOCONV and not raise_noconv:
            return HIterResult(total, st.unconverged, False, nl, rho, nnb, moved)
        ctx.check(rc)
        return HIterResult(total, st.unconverged, True, nl, rho, nnb, moved)


# --------------------------------------------------------------------------
# Learned h-seed: the MLP and its training (sfcnl_mlp_*, sfcnl_hseed_features)
# --------------------------------------------------------------------------

MLP_NPARAM = _lib.MLP_NPARAM


def hseed_features(ctx: Context, keys, x, y, z, h, nnb, box_edge: float, target: int, feat=None):
    """Seed features (bf16 bits, [n, 8]); nnb None: no count yet."""
    n = h.numel()
    feat = ctx.empty((max(n, 1), _lib.HSEED_NFEAT), torch.int16) if feat is None else feat
    ctx.check(ctx.lib.sfcnl_hseed_features(ctx.handle, n, _ptr(keys), _ptr(x), _ptr(y), _ptr(z), _ptr(h), _ptr(nnb),
                                           box_edge, target, _ptr(feat)))
    return feat


def mlp_init(ctx: Context, seed: int = 1):
    p = ctx.empty(MLP_NPARAM, torch.float32)
    ctx.check(ctx.lib.sfcnl_mlp_init(ctx.handle, seed, _ptr(p)))
    return p


def mlp_infer(ctx: Context, params, feat, out=None):
    n = feat.shape[0]
    out = ctx.empty(max(n, 1), torch.float32) if out is None else out
    ctx.check(ctx.lib.sfcnl_mlp_infer(ctx.handle, _ptr(params), n, _ptr(feat), _ptr(out)))
    return out


def mlp_grad(ctx: Context, params, feat, target, batch: int, start: int = 0, mul: int = 1, add: int = 0,
             ws=None, grad=None, loss=None):
    nsamp = feat.shape[0]
    b = C.c_size_t()
    ctx.lib.sfcnl_mlp_grad_workspace(batch, C.byref(b))
    ws = ctx.empty(b.value, torch.uint8) if ws is None or ws.numel() < b.value else ws
    grad = ctx.empty(MLP_NPARAM, torch.float32) if grad is None else grad
    loss = ctx.empty(1, torch.float32) if loss is None else loss
    ctx.check(ctx.lib.sfcnl_mlp_grad(ctx.handle, _ptr(params), nsamp, _ptr(feat), _ptr(target), batch, start, mul,
                                     add, _ptr(ws), ws.numel(), _ptr(grad), _ptr(loss)))
    return grad, loss, ws


def mlp_adam(ctx: Context, params, grad, m, v, t: int, lr: float):
    ctx.check(ctx.lib.sfcnl_mlp_adam(ctx.handle, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), t, lr))


def _coprime_multiplier(n: int) -> int:
    import math
    mul = 2654435761  # a prime near 2^32 / golden ratio
    while math.gcd(mul, n) != 1:
        mul += 2
    return mul


def mlp_train(ctx: Context, feat, target, epochs: int = 30, batch: int = 8192, lr: float = 3e-3,
              lr_final: float = 3e-4, seed: int = 1, params=None, log=None):
    """Trains the seed MLP with the library's kernels (gradient + Adam per
    batch, samples visited in a fresh permutation every epoch). Returns
    (params, losses per epoch)."""
    n = feat.shape[0]
    params = mlp_init(ctx, seed) if params is None else params
    m = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=params.device)
    v = torch.zeros_like(m)
    mul = _coprime_multiplier(n)
    steps = max(1, n // batch)
    grad, loss, ws = None, None, None
    losses = []
    t = 0
    for ep in range(epochs):
        acc = 0.0
        for k in range(steps):
            t += 1
            frac = (t - 1) / max(1, epochs * steps - 1)
            lr_t = lr * (lr_final / lr) ** frac
            grad, loss, ws = mlp_grad(ctx, params, feat, target, batch, start=k * batch, mul=mul,
                                      add=(ep * 7919) % n, ws=ws, grad=grad, loss=loss)
            mlp_adam(ctx, params, grad, m, v, t, lr_t)
            if k == steps - 1 or k % 32 == 0:
                acc = float(loss.item())
        losses.append(acc)
        if log:
            log("epoch %d loss %.5f" % (ep, acc))
    return params, losses


class Pipeline:
    """The whole path on one system with every buffer preallocated:
    sfc_sort -> sfc_gather -> build_clusters -> build_nlist -> nlist_pass."""

    def __init__(self, ctx: Context, n: int, box, compress: bool = True, leaf_bucket: int = 128,
                 max_j_per_sc: int = 256, with_mass: bool = False, cluster_size: int = CLUSTER_SIZE,
                 half: bool = False, period=None):
        self.ctx, self.n, self.box = ctx, n, tuple(float(v) for v in box)
        self.period = _period(period)
        self.compress, self.leaf_bucket, self.max_j_per_sc = compress, leaf_bucket, max_j_per_sc
        self.cluster_size, self.half = cluster_size, half
        nsc = (n + SC_SIZE - 1) // SC_SIZE
        nc = (n + cluster_size - 1) // cluster_size
        e = ctx.empty
        self.keys, self.perm = e(max(n, 1), torch.int64), e(max(n, 1), torch.int32)
        self.sort_ws = e(max(sfc_sort_workspace(n), 1), torch.uint8)
        self.gather_ws = e(max(sfc_gather_workspace(n), 1), torch.uint8)
        nf = 5 if with_mass else 4
        self.sorted = [e(max(n, 1), torch.float32) for _ in range(nf)]
        self.bbox = e((max(nc, 1), 8), torch.float32)
        self.sc_info = e((max(nsc, 1), 2), torch.int32)
        self.pool = e(max(1024, 6 * n), torch.int32)
        self.ws = e(max(build_nlist_workspace(n, cluster_size, compress, leaf_bucket, max_j_per_sc), 1), torch.uint8)
        self.rho, self.nnb = e(max(n, 1), torch.float32), e(max(n, 1), torch.int32)
        self.nl = None

    def step(self, x, y, z, h, m=None, want_counts=True, density=True):
        """One pass of the path; density=False stops after the list build.
        Once a build has fixed the buffer sizes, later steps enqueue the pass
        right behind the build and check the build's status afterwards
        (build_nlist_async), redoing both if the list outgrew its buffers."""
        ctx, n = self.ctx, self.n
        sfc_sort(ctx, x, y, z, self.box, self.keys, self.perm, self.sort_ws)
        fields = [x, y, z, h] + ([m] if m is not None else [])
        outs = self.sorted[:len(fields)]
        sfc_gather(ctx, self.perm, fields, outs, ws=self.gather_ws)
        xs, ys, zs, hs = outs[:4]
        ms = outs[4] if m is not None else None
        build_clusters(ctx, xs, ys, zs, hs, self.cluster_size, self.bbox)
        if self.nl is not None and density:
            nl = build_nlist_async(ctx, self.keys, xs, ys, zs, hs, self.bbox, self.pool, self.ws, self.sc_info,
                                   self.compress, self.leaf_bucket, self.max_j_per_sc, self.cluster_size,
                                   self.half, self.period)
            nlist_pass(ctx, nl, xs, ys, zs, hs, ms, self.rho, self.nnb if want_counts else None, want_counts)
            if build_nlist_finish(ctx, nl):
                self.nl = nl
                return nl
        nl = build_nlist(ctx, self.keys, xs, ys, zs, hs, self.bbox, self.compress, self.leaf_bucket,
                         self.max_j_per_sc, self.cluster_size, pool=self.pool, ws=self.ws, sc_info=self.sc_info,
                         half=self.half, period=self.period)
        if nl.pool is not self.pool or nl.ws is not self.ws:  # grown on a retry: keep the larger buffers
            self.pool, self.ws, self.max_j_per_sc = nl.pool, nl.ws, nl.max_j_per_sc
        self.nl = nl
        if density:
            nlist_pass(ctx, nl, xs, ys, zs, hs, ms, self.rho, self.nnb if want_counts else None, want_counts)
        return nl


# --------------------------------------------------------------------------
# Batches of independent systems (sfcnl_batch_*)
# --------------------------------------------------------------------------

class Batch:
    """sfcnl_batch_create: a batch of systems with the given particle counts
    and key boxes (6 floats each) on the context's device."""

    def __init__(self, ctx: Context, counts, boxes):
        import numpy as np
        self.ctx = ctx
        counts = np.ascontiguousarray(np.asarray(counts, dtype=np.int64))
        boxes = np.ascontiguousarray(np.asarray(boxes, dtype=np.float32).reshape(-1))
        self.nsys = int(counts.size)
        if boxes.size != 6 * self.nsys:
            raise ValueError("need 6 box values per system")
        h = C.c_void_p()
        ctx.check(ctx.lib.sfcnl_batch_create(ctx.handle, self.nsys, counts.ctypes.data_as(C.POINTER(C.c_int64)),
                                             boxes.ctypes.data_as(C.POINTER(C.c_float)), C.byref(h)))
        self.handle = h
        n_in, n_pad = C.c_int64(), C.c_int64()
        self.in_off = np.zeros(self.nsys + 1, dtype=np.int64)
        self.pbase = np.zeros(self.nsys + 1, dtype=np.int64)
        ctx.check(ctx.lib.sfcnl_batch_layout(h, C.byref(n_in), C.byref(n_pad),
                                             self.in_off.ctypes.data_as(C.POINTER(C.c_int64)),
                                             self.pbase.ctypes.data_as(C.POINTER(C.c_int64))))
        self.n_in, self.n_pad = n_in.value, n_pad.value
        self.counts = counts

    def close(self):
        if getattr(self, "handle", None):
            self.ctx.lib.sfcnl_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sc_range(self, s: int):
        return int(self.pbase[s]) // SC_SIZE, int(self.pbase[s + 1]) // SC_SIZE


def batch_create(ctx: Context, counts, boxes) -> Batch:
    return Batch(ctx, counts, boxes)


def batch_sort(ctx: Context, b: Batch, x, y, z, keys=None, perm=None, ws=None):
    """(keys int64 view of u64, perm int32 view of u32), both padded."""
    wsb = C.c_size_t()
    ctx.check(ctx.lib.sfcnl_batch_sort_workspace(b.handle, C.byref(wsb)))
    keys = ctx.empty(max(b.n_pad, 1), torch.int64) if keys is None else keys
    perm = ctx.empty(max(b.n_pad, 1), torch.int32) if perm is None else perm
    ws = ctx.empty(max(wsb.value, 1), torch.uint8) if ws is None else ws
    for t, nm in ((x, "x"), (y, "y"), (z, "z")):
        _check_f32(t, b.n_in, nm)
    ctx.check(ctx.lib.sfcnl_batch_sort(ctx.handle, b.handle, _ptr(x), _ptr(y), _ptr(z), _ptr(keys), _ptr(perm),
                                       _ptr(ws), ws.numel()))
    return keys, perm


def batch_gather(ctx: Context, b: Batch, perm, fields, outs=None):
    nf = len(fields)
    outs = [ctx.empty(max(b.n_pad, 1), torch.float32) for _ in range(nf)] if outs is None else outs
    for f in fields:
        _check_f32(f, b.n_in, "field")
    ins = (C.c_void_p * nf)(*[f.data_ptr() for f in fields])
    out = (C.c_void_p * nf)(*[o.data_ptr() for o in outs])
    ctx.check(ctx.lib.sfcnl_batch_gather(ctx.handle, b.handle, _ptr(perm), nf, ins, out))
    return outs


def batch_build_clusters(ctx: Context, b: Batch, x, y, z, h, bbox=None, cluster_size: int = CLUSTER_SIZE):
    nc = (b.n_pad + cluster_size - 1) // cluster_size
    bbox = ctx.empty((max(nc, 1), 8), torch.float32) if bbox is None else bbox
    if bbox.numel() < 8 * nc:
        raise ValueError("bbox holds %d boxes, %d clusters need them" % (bbox.numel() // 8, nc))
    ctx.check(ctx.lib.sfcnl_batch_build_clusters(ctx.handle, b.handle, _ptr(x), _ptr(y), _ptr(z), _ptr(h),
                                                 cluster_size, _ptr(bbox)))
    return bbox


def batch_nlist_workspace(b: Batch, compress=True, leaf_bucket=128, max_j_per_sc=256,
                          cluster_size: int = CLUSTER_SIZE, half: bool = False) -> int:
    out = C.c_size_t()
    o = _opts(cluster_size, compress, leaf_bucket, max_j_per_sc, half)
    if _lib.load().sfcnl_batch_nlist_workspace(b.handle, C.byref(o), C.byref(out)) != 0:
        raise SfcnlError(_lib.E_ARG, "sfcnl_batch_nlist_workspace")
    return out.value


def batch_build_nlist(ctx: Context, b: Batch, keys, x, y, z, h, bbox, compress: bool = True, leaf_bucket: int = 128,
                      max_j_per_sc: int = 256, pool=None, ws=None, sc_info=None, grow: bool = True,
                      cluster_size: int = CLUSTER_SIZE, half: bool = False):
    """The padded batch's list (one pool, sc_info per padded super-cluster)."""
    n = b.n_pad
    nsc = n // SC_SIZE
    sc_info = ctx.empty((max(nsc, 1), 2), torch.int32) if sc_info is None else sc_info
    pool = ctx.empty(max(1024, 5 * n), torch.int32) if pool is None else pool
    while True:
        o = _opts(cluster_size, compress, leaf_bucket, max_j_per_sc, half)
        need = batch_nlist_workspace(b, compress, leaf_bucket, max_j_per_sc, cluster_size, half)
        if ws is None or ws.numel() < need:
            ws = ctx.empty(max(need, 1), torch.uint8)
        used, maxnj = C.c_size_t(), C.c_int64()
        rc = ctx.lib.sfcnl_batch_build_nlist(ctx.handle, b.handle, _ptr(keys), _ptr(x), _ptr(y), _ptr(z), _ptr(h),
                                             _ptr(bbox), C.byref(o), _ptr(ws), ws.numel(), _ptr(sc_info), _ptr(pool),
                                             pool.numel() * 4, C.byref(used), C.byref(maxnj))
        if rc == _lib.E_CAPACITY and grow:
            grown = False
            if maxnj.value > max_j_per_sc:
                max_j_per_sc = int(maxnj.value)
                grown = True
            if used.value > pool.numel() * 4:
                pool = ctx.empty(used.value // 4 + 1024, torch.int32)
                grown = True
            if not grown:  # the reported sizes already held: retrying would not change anything
                ctx.check(rc)
            continue
        ctx.check(rc)
        nl = NeighbourList(n, cluster_size, bool(compress), sc_info[:nsc], pool, used.value, maxnj.value,
                           bool(half))
        nl.ws, nl.max_j_per_sc = ws, max_j_per_sc
        return nl


def batch_pass(ctx: Context, b: Batch, nl: NeighbourList, x, y, z, h, m=None, rho=None, nnb=None):
    n = b.n_pad
    rho = ctx.empty(max(n, 1), torch.float32) if rho is None else rho
    nnb = ctx.empty(max(n, 1), torch.int32) if nnb is None else nnb
    ctx.check(ctx.lib.sfcnl_batch_pass(ctx.handle, b.handle, nl.cluster_size, int(nl.compress), int(nl.half),
                                       _ptr(nl.sc_info),
                                       _ptr(nl.pool), _ptr(x), _ptr(y), _ptr(z), _ptr(h), _ptr(m), _ptr(rho),
                                       _ptr(nnb)))
    return rho, nnb


@dataclass
class BatchIterResult:
    iters: int
    unconverged: int
    converged: bool
    sys_rounds: "object"  # numpy int32 [nsys]
    moved: int
    used_bytes: int
    rho: torch.Tensor
    nnb: torch.Tensor

    def mean_rounds(self, n_real: int) -> float:
        return self.moved / max(n_real, 1) + 1.0


def batch_h_iterate(ctx: Context, b: Batch, keys, x, y, z, h, target: int = 100, tol: int = 1, max_iters: int = 64,
                    m=None, compress: bool = True, leaf_bucket: int = 128, max_j_per_sc: int = 256,
                    use_graph: bool = True, mlp_params=None, seed_mode: int = _lib.SEED_AFTER_FIRST,
                    bufs: dict | None = None, cluster_size: int = CLUSTER_SIZE, half: bool = False,
                    recount: int = 0):
    """sfcnl_batch_h_iterate on padded SFC-ordered arrays (h updated in
    place). `bufs` (a dict, filled on first use) keeps every buffer for reuse
    across calls; buffers grow and the run resumes on SFCNL_E_CAPACITY.
    recount: 0 automatic, 1 lists, 2 one wavefront per moved particle."""
    import numpy as np
    n = b.n_pad
    nsc = n // SC_SIZE
    nc = n // cluster_size
    e = ctx.empty
    B = {} if bufs is None else bufs
    if "bracket" not in B:
        B["bracket"] = e(max(2 * n, 2), torch.float32)
        B["bbox"] = e((max(nc, 1), 8), torch.float32)
        B["sc_info"] = e((max(nsc, 1), 2), torch.int32)
        B["pool"] = e(max(1024, 6 * n), torch.int32)
        B["rho"] = e(max(n, 1), torch.float32)
        B["nnb"] = e(max(n, 1), torch.int32)
    B.setdefault("max_j", max_j_per_sc)
    if B["bbox"].numel() < 8 * nc:  # a smaller cluster size needs more boxes
        B["bbox"] = e((max(nc, 1), 8), torch.float32)
    hs = None
    if mlp_params is not None:
        if "feat" not in B:
            B["feat"] = e((max(n, 1), _lib.HSEED_NFEAT), torch.int16)
            B["delta"] = e(max(n, 1), torch.float32)
        hs = _lib.HSeed(mlp_params.data_ptr(), B["feat"].data_ptr(), B["delta"].data_ptr(), 0.0, seed_mode)
    rounds = np.zeros(b.nsys, dtype=np.int32)
    total, moved, resume = 0, 0, 0
    while True:
        mj = B["max_j"]
        need = batch_nlist_workspace(b, compress, leaf_bucket, mj, cluster_size, half)
        if "ws" not in B or B["ws"].numel() < need:
            B["ws"] = e(max(need, 1), torch.uint8)
        no = _opts(cluster_size, compress, leaf_bucket, mj, half)
        io = _lib.HiterOpts(target, tol, max(max_iters - total, 1), resume, int(recount))
        st = _lib.HiterStats()
        r = np.zeros(b.nsys, dtype=np.int32)
        seed_arg = C.byref(hs) if (hs is not None and total == 0) else None
        rc = ctx.lib.sfcnl_batch_h_iterate(ctx.handle, b.handle, _ptr(keys), _ptr(x), _ptr(y), _ptr(z), _ptr(h),
                                           _ptr(B["bracket"]), _ptr(m), C.byref(no), C.byref(io), _ptr(B["bbox"]),
                                           _ptr(B["ws"]), B["ws"].numel(), _ptr(B["sc_info"]), _ptr(B["pool"]),
                                           B["pool"].numel() * 4, _ptr(B["rho"]), _ptr(B["nnb"]), seed_arg,
                                           int(bool(use_graph)), C.byref(st), r.ctypes.data_as(C.POINTER(C.c_int32)))
        rounds = np.where(r > 0, total + r, rounds)
        total += st.iters
        moved += st.moved
        if rc == _lib.E_CAPACITY:
            if st.max_nj > mj:
                B["max_j"] = int(st.max_nj)
            if st.used_bytes > B["pool"].numel() * 4:
                B["pool"] = e(st.used_bytes // 4 + 1024, torch.int32)
            if st.unconverged == 0 and st.iters > 0:
                # converged, only the closing list did not fit: build it with room
                batch_build_clusters(ctx, b, x, y, z, h, B["bbox"], cluster_size)
                nl = batch_build_nlist(ctx, b, keys, x, y, z, h, B["bbox"], compress, leaf_bucket, B["max_j"],
                                       pool=B["pool"], ws=B["ws"], sc_info=B["sc_info"], cluster_size=cluster_size,
                                       half=half)
                B["pool"], B["max_j"] = nl.pool, nl.max_j_per_sc
                return BatchIterResult(total, 0, True, rounds, moved, nl.used_bytes, B["rho"], B["nnb"])
            resume = 1
            continue
        conv = rc == 0
        if rc not in (0, _lib.E_NOCONV):
            ctx.check(rc)
        return BatchIterResult(total, st.unconverged, conv, rounds, moved, st.used_bytes, B["rho"], B["nnb"])
