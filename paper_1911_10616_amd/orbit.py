"""Thin Python binding of liborbit_hip.so (argument marshalling only).

Every step of the counting runs in the library's HIP kernels; PyTorch only
provides device memory and the current HIP stream.  Importing this module
loads the library and fails loudly if it has not been built.
"""
from __future__ import annotations

import contextlib
import ctypes
import os

import numpy as np

from .build import LIB, LIB_TILES

NORB = 73
ORB_NONINDUCED = 0x1
ORB_TIMING = 0x2
ORB_RELABEL = 0x4
ORB_SERIAL_GROUPS = 0x8
ORB_ASYNC = 0x10
SCHED_ID, SCHED_STATIC, SCHED_MLP = 0, 1, 2
SCHEDULES = {"id": SCHED_ID, "static": SCHED_STATIC, "mlp": SCHED_MLP}
GROUPS = {"auto": 0, "wg": 1, "wave": 2}
MLP_PARAMS = 1217

EXPORTS = ("orbit_num_orbits", "orbit_count", "orbit_workspace_query", "orbit_count_ex",
           "orbit_strerror", "orbit_last_phase_times", "orbit_last_stats", "orbit_mlp_init",
           "orbit_mlp_predict", "orbit_mlp_grad", "orbit_mlp_train", "orbit_count_batched",
           "orbit_workspace_query_batched", "orbit_autotune", "orbit_plan_create",
           "orbit_plan_launch", "orbit_plan_status", "orbit_plan_destroy",
           "orbit_count_noalloc", "orbit_noalloc_capacity", "orbit_count_edges",
           "orbit_num_patterns", "orbit_voc_summary", "orbit_last_kernel_times",
           "orbit_prepare", "orbit_count_status")


class OrbError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status} ({_lib.orbit_strerror(status).decode()})")


class _Opts(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("num_wg", ctypes.c_uint32),
                ("schedule", ctypes.c_uint32), ("groups", ctypes.c_uint32),
                ("mlp_weights", ctypes.c_void_p), ("features_out", ctypes.c_void_p),
                ("steps_out", ctypes.c_void_p), ("pass_cycles_out", ctypes.c_void_p),
                ("sizes", ctypes.c_void_p)]


class _Sizes(ctypes.Structure):
    _fields_ = [("ntri", ctypes.c_uint64), ("peel_groups", ctypes.c_uint32),
                ("maxlevel", ctypes.c_uint32), ("gmax", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


def _load(path=LIB):
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_1911_10616_amd.build.build()")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    u64 = ctypes.c_uint64
    lib.orbit_num_orbits.argtypes = [ctypes.c_int]
    lib.orbit_num_orbits.restype = ctypes.c_int
    lib.orbit_count.argtypes = [vp, vp, ctypes.c_uint32, u64, ctypes.c_int, vp]
    lib.orbit_count.restype = ctypes.c_int
    lib.orbit_workspace_query.argtypes = [vp, vp, ctypes.c_uint32, u64, ctypes.c_int, vp,
                                          ctypes.POINTER(_Opts), ctypes.POINTER(u64)]
    lib.orbit_workspace_query.restype = ctypes.c_int
    lib.orbit_count_ex.argtypes = [vp, vp, ctypes.c_uint32, u64, ctypes.c_int, vp, vp, vp, u64,
                                   ctypes.POINTER(u64), vp, ctypes.POINTER(_Opts)]
    lib.orbit_count_ex.restype = ctypes.c_int
    lib.orbit_strerror.argtypes = [ctypes.c_int]
    lib.orbit_strerror.restype = ctypes.c_char_p
    lib.orbit_last_phase_times.argtypes = [ctypes.POINTER(ctypes.c_float),
                                           ctypes.POINTER(ctypes.c_char_p), ctypes.c_int]
    lib.orbit_last_phase_times.restype = ctypes.c_int
    lib.orbit_last_kernel_times.argtypes = [ctypes.POINTER(ctypes.c_float),
                                            ctypes.POINTER(ctypes.c_char_p), ctypes.c_int]
    lib.orbit_last_kernel_times.restype = ctypes.c_int
    lib.orbit_last_stats.argtypes = [ctypes.POINTER(u64), ctypes.c_int]
    lib.orbit_last_stats.restype = ctypes.c_int
    lib.orbit_mlp_init.argtypes = [vp, ctypes.c_uint32, vp]
    lib.orbit_mlp_init.restype = ctypes.c_int
    lib.orbit_mlp_predict.argtypes = [vp, vp, ctypes.c_uint32, vp, vp]
    lib.orbit_mlp_predict.restype = ctypes.c_int
    lib.orbit_mlp_grad.argtypes = [vp, vp, vp, vp, ctypes.c_uint32, vp, vp, vp]
    lib.orbit_mlp_grad.restype = ctypes.c_int
    lib.orbit_mlp_train.argtypes = [vp, vp, ctypes.c_uint32, vp, vp, ctypes.c_uint32,
                                    ctypes.c_uint32, ctypes.c_float, ctypes.c_uint32, vp]
    lib.orbit_mlp_train.restype = ctypes.c_int
    u32 = ctypes.c_uint32
    lib.orbit_count_batched.argtypes = [vp, u32, vp, vp, u32, u64, ctypes.c_int, vp, vp, u64,
                                        ctypes.POINTER(u64), vp, ctypes.POINTER(_Opts)]
    lib.orbit_count_batched.restype = ctypes.c_int
    lib.orbit_workspace_query_batched.argtypes = [vp, u32, vp, vp, u32, u64, ctypes.c_int, vp,
                                                  ctypes.POINTER(_Opts), ctypes.POINTER(u64)]
    lib.orbit_workspace_query_batched.restype = ctypes.c_int
    lib.orbit_autotune.argtypes = [vp, u32, vp, vp, u32, u64, ctypes.c_int, vp, vp, u64, vp,
                                   ctypes.POINTER(_Opts), ctypes.POINTER(u32), ctypes.c_int,
                                   ctypes.POINTER(_Opts), ctypes.POINTER(ctypes.c_float)]
    lib.orbit_autotune.restype = ctypes.c_int
    lib.orbit_plan_create.argtypes = [vp, u32, vp, vp, u32, u64, ctypes.c_int, vp, vp, u64, vp,
                                      ctypes.POINTER(_Opts), ctypes.POINTER(vp)]
    lib.orbit_plan_create.restype = ctypes.c_int
    for f in (lib.orbit_plan_launch, lib.orbit_plan_status):
        f.argtypes = [vp, vp]
        f.restype = ctypes.c_int
    lib.orbit_plan_destroy.argtypes = [vp]
    lib.orbit_plan_destroy.restype = ctypes.c_int
    lib.orbit_count_edges.argtypes = [vp, vp, u32, u64, ctypes.c_int, vp, vp, vp, u64,
                                      ctypes.POINTER(u64), vp, ctypes.POINTER(_Opts)]
    lib.orbit_count_edges.restype = ctypes.c_int
    lib.orbit_prepare.argtypes = [vp, vp, u32, u64, ctypes.c_int, vp, ctypes.POINTER(_Opts),
                                  ctypes.POINTER(u64), ctypes.POINTER(_Sizes)]
    lib.orbit_prepare.restype = ctypes.c_int
    lib.orbit_count_status.argtypes = [vp, vp]
    lib.orbit_count_status.restype = ctypes.c_int
    lib.orbit_num_patterns.argtypes = [ctypes.c_int]
    lib.orbit_num_patterns.restype = ctypes.c_int
    lib.orbit_voc_summary.argtypes = [vp, u32, ctypes.c_int, vp, vp, vp, vp]
    lib.orbit_voc_summary.restype = ctypes.c_int
    lib.orbit_count_noalloc.argtypes = [vp, vp, u32, u64, ctypes.c_int, vp, vp]
    lib.orbit_count_noalloc.restype = ctypes.c_int
    lib.orbit_noalloc_capacity.argtypes = []
    lib.orbit_noalloc_capacity.restype = u64
    return lib


_lib = _load()
_loaded = {LIB: _lib}


@contextlib.contextmanager
def using_library(path=LIB_TILES):
    """Route every call of this module to another build of the library
    (the tests use the small-tile build) inside the with-block."""
    global _lib
    if path not in _loaded:
        _loaded[path] = _load(path)
    old = _lib
    _lib = _loaded[path]
    try:
        yield
    finally:
        _lib = old


def num_orbits(k_max: int) -> int:
    return _lib.orbit_num_orbits(k_max)


def _dev_csr(row_ptr, col_idx, device="cuda"):
    import torch
    rp = torch.as_tensor(np.asarray(row_ptr, dtype=np.uint32).view(np.int32)) \
        if not isinstance(row_ptr, torch.Tensor) else row_ptr
    ci = torch.as_tensor(np.asarray(col_idx, dtype=np.uint32).view(np.int32)) \
        if not isinstance(col_idx, torch.Tensor) else col_idx
    rp = rp.to(device).contiguous()
    ci = ci.to(device).contiguous()
    if ci.numel() == 0:
        ci = torch.zeros(1, dtype=torch.int32, device=device)
    return rp, ci


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _opts(noninduced=False, timing=False, num_wg=0, schedule=SCHED_ID, mlp_weights=None,
          features_out=None, steps_out=None, groups=0, pass_cycles_out=None, relabel=False,
          serial=False):
    f = (ORB_NONINDUCED if noninduced else 0) | (ORB_TIMING if timing else 0) | \
        (ORB_RELABEL if relabel else 0) | (ORB_SERIAL_GROUPS if serial else 0)
    g = GROUPS[groups] if isinstance(groups, str) else int(groups)
    return _Opts(f, num_wg, schedule, g, _ptr(mlp_weights), _ptr(features_out), _ptr(steps_out),
                 _ptr(pass_cycles_out))


def workspace_bytes(row_ptr, col_idx, k_max=5, noninduced=False, num_wg=0, stream=None,
                    groups="auto", relabel=False) -> int:
    rp, ci = _dev_csr(row_ptr, col_idx)
    n = rp.numel() - 1
    m = int(rp[-1].item()) // 2 if n >= 0 else 0
    out = ctypes.c_uint64(0)
    o = _opts(noninduced, False, num_wg, groups=groups, relabel=relabel)
    st = _lib.orbit_workspace_query(ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(ci.data_ptr()),
                                    n, m, k_max, _stream_ptr(stream), ctypes.byref(o),
                                    ctypes.byref(out))
    if st:
        raise OrbError(st, "orbit_workspace_query")
    return int(out.value)


class Counter:
    """Counts orbits of one graph repeatedly with a workspace allocated once.

    row_ptr/col_idx: symmetric CSR (uint32 values; numpy arrays or int32
    torch tensors holding the same bits).  Results are uint64 counts
    returned as an int64 torch tensor of shape [n, K] holding the same bits
    (use ``.cpu().numpy().view(np.uint64)``)."""

    def __init__(self, row_ptr, col_idx, k_max=5, noninduced=False, num_wg=0, stream=None,
                 schedule="id", mlp_weights=None, features_out=None, steps_out=None,
                 groups="auto", pass_cycles_out=None, relabel=False, serial=False,
                 asynchronous=False):
        """schedule: "id", "static" or "mlp" (source order of the per-source
        kernels; needs mlp_weights, a float32 device tensor of MLP_PARAMS
        values, for "mlp").  features_out (float32 [n, 3]) and steps_out
        (int64 [n], uint64 bits) receive the cost features and per-source
        pair-sweep step counts on every run when given; pass_cycles_out (int64
        [4]) accumulates the pair sweep's per-pass clock cycles.  relabel=True
        counts on a copy renumbered heaviest degree class first (ORB_RELABEL)."""
        import torch
        self.rp, self.ci = _dev_csr(row_ptr, col_idx)
        self.n = self.rp.numel() - 1
        self.m = int(self.rp[-1].item()) // 2
        self.k_max = k_max
        self.K = num_orbits(k_max)
        if not self.K:
            raise OrbError(-1, "k_max")
        sched = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
        extra = dict(schedule=sched, mlp_weights=mlp_weights, features_out=features_out,
                     steps_out=steps_out, groups=groups, pass_cycles_out=pass_cycles_out,
                     relabel=relabel, serial=serial)
        self._keep = (mlp_weights, features_out, steps_out, pass_cycles_out)
        self.opts = _opts(noninduced, False, num_wg, **extra)
        self.topts = _opts(noninduced, True, num_wg, **extra)
        self.stream = stream
        self.sizes = None
        if asynchronous:
            # orbit_prepare: the sizes of this graph's count (synchronises
            # once); run() then enqueues with no host synchronisation
            self.sizes = _Sizes()
            need = ctypes.c_uint64(0)
            _check(_lib.orbit_prepare(ctypes.c_void_p(self.rp.data_ptr()),
                                      ctypes.c_void_p(self.ci.data_ptr()), self.n, self.m, k_max,
                                      _stream_ptr(stream), ctypes.byref(self.opts),
                                      ctypes.byref(need), ctypes.byref(self.sizes)),
                   "orbit_prepare")
            self.ws_bytes = int(need.value)
            for o in (self.opts, self.topts):
                o.flags |= ORB_ASYNC
                o.sizes = ctypes.cast(ctypes.pointer(self.sizes), ctypes.c_void_p)
        else:
            self.ws_bytes = workspace_bytes(self.rp, self.ci, k_max, noninduced, num_wg, stream,
                                            groups=groups, relabel=relabel)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.rp.device)
        self.out = torch.empty((max(self.n, 1), self.K), dtype=torch.int64, device=self.rp.device)

    def status(self):
        """orbit_count_status: waits for the stream and raises if the last
        count recorded an error (the check of asynchronous counts)."""
        _check(_lib.orbit_count_status(ctypes.c_void_p(self.ws.data_ptr()),
                                       _stream_ptr(self.stream)), "orbit_count_status")

    def run(self, timing=False, overflow_flags=None):
        """Counts into self.out; overflow_flags: optional uint8 device tensor
        of n entries that receives the overflow flags (1 = the row may have
        wrapped modulo 2^64)."""
        need = ctypes.c_uint64(0)
        o = self.topts if timing else self.opts
        st = _lib.orbit_count_ex(ctypes.c_void_p(self.rp.data_ptr()),
                                 ctypes.c_void_p(self.ci.data_ptr()), self.n, self.m, self.k_max,
                                 ctypes.c_void_p(self.out.data_ptr()), _ptr(overflow_flags),
                                 ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                 ctypes.byref(need), _stream_ptr(self.stream), ctypes.byref(o))
        if st:
            raise OrbError(st, "orbit_count_ex")
        return self.out[: self.n]


def count(row_ptr, col_idx, k_max=5, noninduced=False, num_wg=0, groups="auto",
          relabel=False, overflow_flags=None, serial=False):
    """Orbit counts of one graph as a torch tensor [n, K] on the GPU: int64
    holding the uint64 bits (induced unless noninduced=True).  overflow_flags:
    optional uint8 device tensor [n] for the overflow flags."""
    c = Counter(row_ptr, col_idx, k_max, noninduced, num_wg, groups=groups, relabel=relabel,
                serial=serial)
    return c.run(overflow_flags=overflow_flags).clone()


def count_edges(row_ptr, col_idx, k_max=4, noninduced=False, groups="auto"):
    """(vertex counts [n, K], edge orbit counts [2m, 12]) as torch tensors
    (int64 holding uint64 bits): orbit_count_edges.  Row s of the edge
    counts is E_0..E_11 of CSR slot s = (u, v), oriented with u in the
    endpoint vertex orbit of larger index."""
    import torch
    c = Counter(row_ptr, col_idx, k_max, noninduced, groups=groups)
    m2 = 2 * c.m
    edges = torch.empty((max(m2, 1), 12), dtype=torch.int64, device=c.rp.device)
    need = ctypes.c_uint64(0)
    _check(_lib.orbit_count_edges(ctypes.c_void_p(c.rp.data_ptr()), ctypes.c_void_p(c.ci.data_ptr()),
                                  c.n, c.m, k_max, ctypes.c_void_p(c.out.data_ptr()),
                                  ctypes.c_void_p(edges.data_ptr()), ctypes.c_void_p(c.ws.data_ptr()),
                                  c.ws_bytes, ctypes.byref(need), _stream_ptr(None),
                                  ctypes.byref(c.opts)), "orbit_count_edges")
    return c.out[:c.n].clone(), edges[:m2]


VOC_BINS = 65


def voc_summary(counts, k_max=5, stream=None):
    """orbit_voc_summary of a count tensor [n, K] on the GPU.  Returns
    (orbit_sums, pattern_counts, hist): Python ints per orbit and per
    pattern (the 128-bit words joined), and a numpy [K, 65] histogram of the
    counts by bit length."""
    import torch
    n = counts.shape[0]
    K = num_orbits(k_max)
    P = _lib.orbit_num_patterns(k_max)
    sums = torch.empty(2 * K, dtype=torch.int64, device=counts.device)
    pats = torch.empty(2 * P, dtype=torch.int64, device=counts.device)
    hist = torch.empty((K, VOC_BINS), dtype=torch.int64, device=counts.device)
    _check(_lib.orbit_voc_summary(ctypes.c_void_p(counts.data_ptr()), n, k_max,
                                  ctypes.c_void_p(sums.data_ptr()), ctypes.c_void_p(pats.data_ptr()),
                                  ctypes.c_void_p(hist.data_ptr()), _stream_ptr(stream)),
           "orbit_voc_summary")
    s = to_u64(sums).reshape(K, 2)
    p = to_u64(pats).reshape(P, 2)
    join = lambda w: [int(a) | (int(b) << 64) for a, b in w]
    return join(s), join(p), to_u64(hist)


def ccd(hist_row, n):
    """Complementary cumulative distribution of one orbit from its
    bit-length histogram: [(x, fraction of vertices with count >= x)] for
    x = 1, 2, 4, ... (the points where the histogram makes it exact)."""
    tail = np.cumsum(np.asarray(hist_row, np.float64)[::-1])[::-1]
    return [(1 << (b - 1), float(tail[b]) / max(n, 1)) for b in range(1, VOC_BINS) if tail[b] > 0]


def to_u64(t) -> np.ndarray:
    """A count tensor as a host numpy uint64 array."""
    return t.cpu().numpy().view(np.uint64)


def count_np(row_ptr, col_idx, k_max=5, **kw) -> np.ndarray:
    """count() copied to the host as uint64[n, K]."""
    return to_u64(count(row_ptr, col_idx, k_max, **kw))


def count_minimal(row_ptr, col_idx, k_max=5) -> np.ndarray:
    """The minimal C entry point orbit_count (internal workspace, null stream)."""
    import torch
    rp, ci = _dev_csr(row_ptr, col_idx)
    n = rp.numel() - 1
    m = int(rp[-1].item()) // 2
    K = num_orbits(k_max)
    out = torch.empty((max(n, 1), K), dtype=torch.int64, device=rp.device)
    torch.cuda.synchronize()
    st = _lib.orbit_count(ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(ci.data_ptr()), n, m,
                          k_max, ctypes.c_void_p(out.data_ptr()))
    if st:
        raise OrbError(st, "orbit_count")
    return out[:n].cpu().numpy().view(np.uint64)


def count_noalloc(row_ptr, col_idx, k_max=5, stream=None):
    """orbit_count_noalloc: the count in the library's static buffer (no
    device allocation inside the call); torch tensor as count()."""
    import torch
    rp, ci = _dev_csr(row_ptr, col_idx)
    n = rp.numel() - 1
    m = int(rp[-1].item()) // 2
    out = torch.empty((max(n, 1), num_orbits(k_max)), dtype=torch.int64, device=rp.device)
    _check(_lib.orbit_count_noalloc(ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(ci.data_ptr()),
                                    n, m, k_max, ctypes.c_void_p(out.data_ptr()),
                                    _stream_ptr(stream)), "orbit_count_noalloc")
    return out[:n]


def last_phase_times():
    ms = (ctypes.c_float * 24)()
    names = (ctypes.c_char_p * 24)()
    k = _lib.orbit_last_phase_times(ms, names, 24)
    return [(names[i].decode(), float(ms[i])) for i in range(k)]


def last_kernel_times():
    """{kernel: ms} of the orbit-group kernels of the last timed call, each
    timed on its own stream."""
    ms = (ctypes.c_float * 8)()
    names = (ctypes.c_char_p * 8)()
    k = _lib.orbit_last_kernel_times(ms, names, 8)
    return {names[i].decode(): float(ms[i]) for i in range(k)}


def last_stats():
    """Work statistics of the last timed call (dict)."""
    v = (ctypes.c_uint64 * 7)()
    k = _lib.orbit_last_stats(v, 7)
    keys = ("n", "m", "triangles", "degeneracy", "wedges", "diamonds", "paths3")
    return {keys[i]: int(v[i]) for i in range(k)}


def _dev_u64(a, device="cuda"):
    import torch
    if isinstance(a, torch.Tensor):
        return a.to(device).contiguous()
    return torch.as_tensor(np.asarray(a, dtype=np.uint64).view(np.int64)).to(device).contiguous()


class BatchCounter:
    """Counts orbits of many small graphs in one call (orbit_count_batched).

    vptr: uint64[B+1] graph offsets; row_ptr/col_idx: the CSR of the
    disjoint union over global ids.  Rows vptr[g]..vptr[g+1]-1 of the
    result are graph g's counts.  Options as for Counter."""

    def __init__(self, vptr, row_ptr, col_idx, k_max=5, noninduced=False, num_wg=0,
                 stream=None, schedule="id", mlp_weights=None, groups="auto"):
        import torch
        self.vptr = _dev_u64(vptr)
        self.B = self.vptr.numel() - 1
        self.rp, self.ci = _dev_csr(row_ptr, col_idx)
        self.n = self.rp.numel() - 1
        self.m = int(self.rp[-1].item()) // 2
        self.k_max = k_max
        self.K = num_orbits(k_max)
        self.stream = stream
        self.noninduced = noninduced
        self._w = mlp_weights
        self.set_options(num_wg, schedule, groups)
        self.out = torch.empty((max(self.n, 1), self.K), dtype=torch.int64, device=self.rp.device)

    def _args(self):
        return (ctypes.c_void_p(self.vptr.data_ptr()), self.B, ctypes.c_void_p(self.rp.data_ptr()),
                ctypes.c_void_p(self.ci.data_ptr()), self.n, self.m, self.k_max)

    def set_options(self, num_wg, schedule, groups="auto"):
        """(Re)size the workspace for these options."""
        import torch
        sched = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
        self.opts = _opts(self.noninduced, False, num_wg, sched, self._w, groups=groups)
        self.topts = _opts(self.noninduced, True, num_wg, sched, self._w, groups=groups)
        need = ctypes.c_uint64(0)
        _check(_lib.orbit_workspace_query_batched(*self._args(), _stream_ptr(self.stream),
                                                  ctypes.byref(self.opts), ctypes.byref(need)),
               "orbit_workspace_query_batched")
        self.ws_bytes = int(need.value)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.rp.device)

    def run(self, timing=False):
        need = ctypes.c_uint64(0)
        o = self.topts if timing else self.opts
        _check(_lib.orbit_count_batched(*self._args(), ctypes.c_void_p(self.out.data_ptr()),
                                        ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                        ctypes.byref(need), _stream_ptr(self.stream),
                                        ctypes.byref(o)), "orbit_count_batched")
        return self.out[: self.n]

    def autotune(self, nwg_candidates=(256, 512, 1024, 2048, 4096)):
        """Pick num_wg, schedule and execution groups by timing each candidate
        (orbit_autotune); keeps the choice and returns (num_wg, schedule,
        groups, gpu_ms)."""
        import torch
        big = max(nwg_candidates)
        self.set_options(big, self.opts.schedule, "wave")
        cand = (ctypes.c_uint32 * len(nwg_candidates))(*nwg_candidates)
        best = _Opts()
        ms = ctypes.c_float(0)
        base = _opts(self.noninduced, False, 0, SCHED_ID, self._w)
        _check(_lib.orbit_autotune(*self._args(), ctypes.c_void_p(self.out.data_ptr()),
                                   ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                   _stream_ptr(self.stream), ctypes.byref(base), cand,
                                   len(nwg_candidates), ctypes.byref(best), ctypes.byref(ms)),
               "orbit_autotune")
        self.set_options(best.num_wg, best.schedule, best.groups)
        return int(best.num_wg), int(best.schedule), int(best.groups), float(ms.value)


class Plan:
    """The whole count of a Counter or BatchCounter captured as one HIP
    graph (orbit_plan_create); launch() replays it into the counter's
    output buffer without any host synchronisation.  The input buffers must
    stay unchanged."""

    def __init__(self, counter):
        self.c = counter
        vptr = getattr(counter, "vptr", None)
        B = getattr(counter, "B", 0)
        h = ctypes.c_void_p(0)
        _check(_lib.orbit_plan_create(
            ctypes.c_void_p(vptr.data_ptr()) if vptr is not None else None, B,
            ctypes.c_void_p(counter.rp.data_ptr()), ctypes.c_void_p(counter.ci.data_ptr()),
            counter.n, counter.m, counter.k_max, ctypes.c_void_p(counter.out.data_ptr()),
            ctypes.c_void_p(counter.ws.data_ptr()), counter.ws_bytes,
            _stream_ptr(counter.stream), ctypes.byref(counter.opts), ctypes.byref(h)),
            "orbit_plan_create")
        self.h = h

    def launch(self):
        _check(_lib.orbit_plan_launch(self.h, _stream_ptr(self.c.stream)), "orbit_plan_launch")
        return self.c.out[: self.c.n]

    def status(self):
        """Waits for the stream; raises if the last replay reported an error."""
        _check(_lib.orbit_plan_status(self.h, _stream_ptr(self.c.stream)), "orbit_plan_status")

    def close(self):
        if self.h:
            _lib.orbit_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def count_batched(vptr, row_ptr, col_idx, k_max=5, noninduced=False, num_wg=0,
                  schedule="id", groups="auto") -> np.ndarray:
    """uint64[n, K]: per-graph counts of a batch, concatenated by graph."""
    c = BatchCounter(vptr, row_ptr, col_idx, k_max, noninduced, num_wg, schedule=schedule,
                     groups=groups)
    return c.run().cpu().numpy().view(np.uint64)


def _check(st, where):
    if st:
        raise OrbError(st, where)


def mlp_init(seed=1, stream=None):
    """Fresh cost-model weights (float32 device tensor of MLP_PARAMS)."""
    import torch
    w = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
    _check(_lib.orbit_mlp_init(w.data_ptr(), seed, _stream_ptr(stream)), "orbit_mlp_init")
    return w


def mlp_predict(weights, features, stream=None):
    import torch
    n = features.shape[0]
    out = torch.empty(max(n, 1), dtype=torch.float32, device=features.device)
    _check(_lib.orbit_mlp_predict(weights.data_ptr(), features.data_ptr(), n, out.data_ptr(),
                                  _stream_ptr(stream)), "orbit_mlp_predict")
    return out[:n]


def mlp_grad(weights, features, targets=None, steps=None, stream=None):
    """(grad [MLP_PARAMS], loss [1]) of the mean squared error over all rows."""
    import torch
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=features.device)
    loss = torch.empty(1, dtype=torch.float32, device=features.device)
    _check(_lib.orbit_mlp_grad(weights.data_ptr(), features.data_ptr(), _ptr(targets),
                               _ptr(steps), features.shape[0], grad.data_ptr(), loss.data_ptr(),
                               _stream_ptr(stream)), "orbit_mlp_grad")
    return grad, loss


def mlp_train(weights, features, steps, iters=300, batch=4096, lr=3e-3, seed=7, stream=None):
    """Adam on log2(1 + steps) targets, weights updated in place; returns
    the last mini-batch loss (synchronises)."""
    import torch
    state = torch.empty(3 * MLP_PARAMS + 1, dtype=torch.float32, device=features.device)
    _check(_lib.orbit_mlp_train(features.data_ptr(), steps.data_ptr(), features.shape[0],
                                weights.data_ptr(), state.data_ptr(), iters, batch, lr, seed,
                                _stream_ptr(stream)), "orbit_mlp_train")
    return float(state[-1].item())


def raw_count_ex(rp, ci, n, m, k_max, counts, ws, ws_bytes, flags=0, stream=None,
                 overflow_flags=None):
    """Direct call of orbit_count_ex with explicit arguments (tests)."""
    need = ctypes.c_uint64(0)
    o = _Opts(flags, 0, 0, 0, None, None, None)
    st = _lib.orbit_count_ex(ctypes.c_void_p(rp), ctypes.c_void_p(ci), n, m, k_max,
                             ctypes.c_void_p(counts), ctypes.c_void_p(overflow_flags),
                             ctypes.c_void_p(ws), ws_bytes,
                             ctypes.byref(need), _stream_ptr(stream), ctypes.byref(o))
    return st, int(need.value)
