"""Python binding of ``libfolty.so`` (include/folty.h), argument marshalling only.

Every step of the query runs in the library's HIP kernels.  If the library is
missing this module raises instead of computing anything itself.  PyTorch is
used only to hand over device memory and streams: inputs may be numpy arrays
(host) or torch tensors (host or device).
"""
from __future__ import annotations

import ctypes
import os
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfolty.so")

OK, EINVAL, ENOTBUILT, ENOMEM, EDEVICE, EOVERFLOW, EBUSY = 0, -1, -2, -3, -4, -5, -6
MEM_HOST, MEM_DEVICE, MEM_DEVICE_BORROWED = 0, 1, 2
DELTA_INF = (1 << 63) - 1
UNIVERSE_DST, UNIVERSE_SRC, UNIVERSE_COMMON = 0, 1, 2
RANK_DEGENERACY, RANK_DEGREE, RANK_RANDOM = 0, 1, 2
QUERY_NO_COUNTS = 1
QUERY_SMALLER_SIDE = 2
QUERY_ONE_PASS = 4
U32_MAX = 0xFFFFFFFF

EXPORTS = (
    "folty_last_error", "folty_version", "folty_load_temporal_graph", "folty_build_index",
    "folty_run_fol_query", "folty_run_fol_query_noalloc", "folty_run_vertex_query", "folty_result_vertices",
    "folty_run_triad_query", "folty_run_triad_query_ws", "folty_result_triads",
    "folty_result_edge_instances",
    "folty_workspace_create", "folty_workspace_free",
    "folty_run_fol_query_ws", "folty_run_batch", "folty_run_multi", "folty_result_pairs",
    "folty_result_counts", "folty_result_stats", "folty_result_free", "folty_graph_stats",
    "folty_graph_vertex_array", "folty_graph_device_bytes", "folty_graph_free",
    "folty_release_cached_memory", "folty_plan_create", "folty_plan_run", "folty_plan_get_info",
    "folty_plan_free", "folty_server_create", "folty_server_submit", "folty_server_poll",
    "folty_server_wait", "folty_server_get_info", "folty_server_destroy",
)


class FoltyError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"folty error {code}: {msg}")
        self.code = code


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class BuildOpts(ctypes.Structure):
    _fields_ = [("rank_mode", ctypes.c_int32), ("cache_triangles", ctypes.c_int32),
                ("rank_seed", ctypes.c_uint64), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_ctx", ctypes.c_void_p)]


def torch_allocator():
    """(alloc, free) callbacks that take the index's device memory from PyTorch's
    caching allocator, on the stream the library names."""
    import torch
    dev = torch.cuda.current_device()

    def alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0))
        except Exception:
            return None

    def free(p, nbytes, stream, ctx):
        torch.cuda.caching_allocator_delete(p)

    return ALLOC_FN(alloc), FREE_FN(free)


class Query(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_int64), ("theta_num", ctypes.c_uint32),
                ("theta_den", ctypes.c_uint32), ("variant", ctypes.c_uint8),
                ("universe", ctypes.c_uint8), ("exclude_other", ctypes.c_uint8),
                ("flags", ctypes.c_uint8)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_jobs", ctypes.c_int32), ("n_queries", ctypes.c_int32), ("items", ctypes.c_int64),
                ("tests", ctypes.c_int64), ("tests_per_chunk", ctypes.c_int32),
                ("temporal_blocks", ctypes.c_int32), ("captured", ctypes.c_int32),
                ("records", ctypes.c_int32), ("last_run_ms", ctypes.c_double),
                ("tune_source", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


INNER_FORALL = 0  # exists u forall_theta v forall_theta2 w
INNER_EXISTS = 1  # exists u forall_theta v exists w


class VertexQuery(ctypes.Structure):
    _fields_ = [("edge", Query), ("theta_num", ctypes.c_uint32), ("theta_den", ctypes.c_uint32),
                ("inner", ctypes.c_uint8), ("reserved", ctypes.c_uint8 * 7)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_int64)]


class ServerInfo(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in (
        "submitted", "completed", "rejected", "queued", "batches", "batched_requests",
        "budget_bytes", "in_use_bytes", "peak_in_use_bytes", "kept_bytes", "peak_concurrent_passes",
        "trimmed_bytes")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in (
        "n", "m_input", "m", "self_loops", "static_edges", "directed_pairs", "max_core",
        "max_out_degree", "wedges", "triangles", "max_multiplicity", "peel_rounds",
        "closing_probes", "enum_items", "batch_size", "tests",
        "n_pairs", "n_certificates")] + [(f, ctypes.c_double) for f in (
            "build_ms", "wedge_ms", "temporal_ms", "threshold_ms", "query_ms", "latency_ms",
            "queue_ms")] + [("filter_passes", ctypes.c_int64), ("core_sweeps", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


TRIAD_TRIPLES, TRIAD_INSTANCES, TRIAD_EDGE_INSTANCES = 1, 2, 4


class TriadQuery(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_int64), ("variant", ctypes.c_uint8), ("flags", ctypes.c_uint8),
                ("reserved", ctypes.c_uint8 * 6)]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FoltyError(EDEVICE, f"{path} is missing: build it with "
                                  "`python -m paper_2507_17215_amd.build_lib`")
    try:
        # torch ships its own HIP runtime under the same soname; loading it first
        # makes libfolty.so bind to that one copy, so torch and the library share
        # one runtime (and one view of the device) in this process
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, I32, I64, PP = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p)
    lib.folty_last_error.restype = ctypes.c_char_p
    lib.folty_version.restype = ctypes.c_char_p
    lib.folty_load_temporal_graph.argtypes = [I32, I64, P, P, P, I32, P, PP]
    lib.folty_build_index.argtypes = [P, ctypes.POINTER(BuildOpts)]
    lib.folty_run_fol_query.argtypes = [P, ctypes.POINTER(Query), PP]
    lib.folty_run_fol_query_noalloc.argtypes = [P, ctypes.POINTER(Query), P, P, P, I64, P, ctypes.POINTER(I64),
                                                ctypes.POINTER(I64)]
    lib.folty_run_vertex_query.argtypes = [P, ctypes.POINTER(VertexQuery), PP]
    lib.folty_result_vertices.argtypes = [P, ctypes.POINTER(I64), PP, PP]
    lib.folty_run_triad_query.argtypes = [P, ctypes.POINTER(TriadQuery), PP]
    lib.folty_run_triad_query_ws.argtypes = [P, ctypes.POINTER(TriadQuery), P, PP]
    lib.folty_result_triads.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64), PP]
    lib.folty_result_edge_instances.argtypes = [P, PP]
    lib.folty_workspace_create.argtypes = [PP]
    lib.folty_workspace_free.argtypes = [P]
    lib.folty_workspace_free.restype = None
    lib.folty_run_fol_query_ws.argtypes = [P, ctypes.POINTER(Query), P, PP]
    lib.folty_run_batch.argtypes = [P, ctypes.POINTER(Query), I32, PP]
    lib.folty_run_multi.argtypes = [PP, ctypes.POINTER(Query), I32, PP]
    lib.folty_result_pairs.argtypes = [P, ctypes.POINTER(I64), PP, PP, PP]
    lib.folty_result_counts.argtypes = [P, ctypes.POINTER(I64), PP]
    lib.folty_result_stats.argtypes = [P, ctypes.POINTER(Stats)]
    lib.folty_result_free.argtypes = [P]
    lib.folty_result_free.restype = None
    lib.folty_graph_stats.argtypes = [P, ctypes.POINTER(Stats)]
    lib.folty_graph_vertex_array.argtypes = [P, I32, P]
    lib.folty_graph_device_bytes.argtypes = [P, ctypes.POINTER(I64)]
    lib.folty_release_cached_memory.argtypes = [ctypes.POINTER(I64)]
    lib.folty_plan_create.argtypes = [PP, I32, ctypes.POINTER(Query), ctypes.POINTER(I32), I32, PP]
    lib.folty_plan_run.argtypes = [P, PP]
    lib.folty_plan_get_info.argtypes = [P, ctypes.POINTER(PlanInfo)]
    lib.folty_plan_free.argtypes = [P]
    lib.folty_plan_free.restype = None
    lib.folty_server_create.argtypes = [ctypes.POINTER(ServerOpts), PP]
    lib.folty_server_submit.argtypes = [P, P, ctypes.POINTER(Query), ctypes.POINTER(I64)]
    lib.folty_server_poll.argtypes = [P, I64, PP]
    lib.folty_server_wait.argtypes = [P, I64, PP]
    lib.folty_server_get_info.argtypes = [P, ctypes.POINTER(ServerInfo)]
    lib.folty_server_destroy.argtypes = [P]
    lib.folty_server_destroy.restype = None
    lib.folty_graph_free.argtypes = [P]
    lib.folty_graph_free.restype = None
    for name in EXPORTS:
        if name not in ("folty_workspace_free", "folty_result_free", "folty_graph_free",
                        "folty_plan_free", "folty_server_destroy", "folty_last_error",
                        "folty_version"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        raise FoltyError(rc, load_library().folty_last_error().decode(errors="replace"))


def to_theta(theta) -> tuple:
    """theta as an exact (num, den): a pair, a Fraction, or a float/str read as a
    decimal and limited to denominators up to 10**6."""
    if isinstance(theta, tuple):
        num, den = theta
    else:
        f = theta if isinstance(theta, Fraction) else Fraction(str(theta)).limit_denominator(10**6)
        num, den = f.numerator, f.denominator
    return int(num), int(den)


def make_query(delta, theta=(1, 2), variant=0, universe=UNIVERSE_DST, exclude_other=False,
               counts=True, smaller_side=False, one_pass=False) -> Query:
    num, den = to_theta(theta)
    if delta is None or delta == float("inf"):
        delta = DELTA_INF
    return Query(int(delta), num, den, int(variant), int(universe), 1 if exclude_other else 0,
                 (0 if counts else QUERY_NO_COUNTS) | (QUERY_SMALLER_SIDE if smaller_side else 0)
                 | (QUERY_ONE_PASS if one_pass else 0))


def _array_arg(x, dtype):
    """(pointer, mem_kind, keepalive) for a numpy array or a torch tensor."""
    try:
        import torch
        if isinstance(x, torch.Tensor):
            want = {np.int32: torch.int32, np.int64: torch.int64}[dtype]
            if x.dtype != want:
                raise TypeError(f"expected {want}, got {x.dtype}")
            x = x.contiguous()
            if x.is_cuda:
                torch.cuda.current_stream(x.device).synchronize()
                return ctypes.c_void_p(x.data_ptr()), MEM_DEVICE, x
            return ctypes.c_void_p(x.data_ptr()), MEM_HOST, x
    except ImportError:
        pass
    a = np.ascontiguousarray(x, dtype=dtype)
    return ctypes.c_void_p(a.ctypes.data), MEM_HOST, a


class Result:
    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle
        lib = load_library()
        n = ctypes.c_int64()
        u, v, c = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib.folty_result_pairs(self._h, ctypes.byref(n), ctypes.byref(u), ctypes.byref(v),
                                      ctypes.byref(c)))
        k = n.value
        self.pair_u = np.ctypeslib.as_array(ctypes.cast(u, ctypes.POINTER(ctypes.c_int32)), (k,)).copy() if k else np.zeros(0, np.int32)
        self.pair_v = np.ctypeslib.as_array(ctypes.cast(v, ctypes.POINTER(ctypes.c_int32)), (k,)).copy() if k else np.zeros(0, np.int32)
        self.n_cert = np.ctypeslib.as_array(ctypes.cast(c, ctypes.POINTER(ctypes.c_uint32)), (k,)).copy() if k else np.zeros(0, np.uint32)
        nc = ctypes.c_int64()
        _check(lib.folty_result_counts(self._h, ctypes.byref(nc), None))
        self.n_certificates = nc.value
        st = Stats()
        _check(lib.folty_result_stats(self._h, ctypes.byref(st)))
        self.stats = st.as_dict()

    def counts(self) -> np.ndarray:
        """Per temporal edge counts in input order (0xFFFFFFFF = self-loop)."""
        lib = load_library()
        p = ctypes.c_void_p()
        _check(lib.folty_result_counts(self._h, None, ctypes.byref(p)))
        m = int(self.stats["m_input"])
        if m == 0:
            return np.zeros(0, np.uint32)
        return np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(ctypes.c_uint32)), (m,)).copy()

    def pairs(self):
        return list(zip(self.pair_u.tolist(), self.pair_v.tolist(), self.n_cert.tolist()))

    def vertices(self):
        """Vertex query: (solution vertices ascending, their qualifying neighbour counts)."""
        n = ctypes.c_int64()
        v, g = ctypes.c_void_p(), ctypes.c_void_p()
        _check(load_library().folty_result_vertices(self._h, ctypes.byref(n), ctypes.byref(v), ctypes.byref(g)))
        k = n.value
        if k == 0:
            return np.zeros(0, np.int32), np.zeros(0, np.uint32)
        return (np.ctypeslib.as_array(ctypes.cast(v, ctypes.POINTER(ctypes.c_int32)), (k,)).copy(),
                np.ctypeslib.as_array(ctypes.cast(g, ctypes.POINTER(ctypes.c_uint32)), (k,)).copy())

    def triads(self) -> dict:
        """Exists-exists-exists result: solution triples (k x 3, sorted by (a, b, w),
        None unless listed), their number, and the temporal triangles (-1 if not counted)."""
        ns, ni, p = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_void_p()
        _check(load_library().folty_result_triads(self._h, ctypes.byref(ns), ctypes.byref(ni),
                                                  ctypes.byref(p)))
        trip = None
        if p.value:
            trip = np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(ctypes.c_int32)),
                                         (ns.value, 3)).copy()
        elif ns.value == 0:
            trip = np.zeros((0, 3), np.int32)
        return dict(n_solutions=ns.value, n_instances=ni.value, triples=trip)

    def edge_instances(self) -> np.ndarray:
        """Temporal triangles per first edge, input order (0 for a self-loop)."""
        p = ctypes.c_void_p()
        _check(load_library().folty_result_edge_instances(self._h, ctypes.byref(p)))
        m = int(self.stats["m_input"])
        if m == 0:
            return np.zeros(0, np.uint64)
        return np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(ctypes.c_uint64)), (m,)).copy()

    def close(self):
        if self._h:
            load_library().folty_result_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Workspace:
    """Scratch memory for one concurrent caller."""

    def __init__(self):
        self._h = ctypes.c_void_p()
        _check(load_library().folty_workspace_create(ctypes.byref(self._h)))

    def close(self):
        if self._h:
            load_library().folty_workspace_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A temporal multigraph resident on the GPU with its query index."""

    def __init__(self, n: int, src, dst, t, stream=None, borrow: bool = False):
        """borrow: device tensors are read in place instead of copied; the graph
        keeps references to them, and the caller must not change them while the
        graph lives."""
        lib = load_library()
        ps, ks, a1 = _array_arg(src, np.int32)
        pd, kd, a2 = _array_arg(dst, np.int32)
        pt, kt, a3 = _array_arg(t, np.int64)
        if not (ks == kd == kt):
            raise ValueError("src, dst and t must all be host or all be device arrays")
        m = int(a1.shape[0])
        if int(a2.shape[0]) != m or int(a3.shape[0]) != m:
            raise ValueError("src, dst and t must have the same length")
        if borrow:
            if ks != MEM_DEVICE:
                raise ValueError("borrow=True needs device tensors")
            ks = MEM_DEVICE_BORROWED
            self._inputs = (a1, a2, a3)
        self._h = ctypes.c_void_p()
        st = ctypes.c_void_p(stream) if stream else None
        _check(lib.folty_load_temporal_graph(int(n), m, ps, pd, pt, ks, st, ctypes.byref(self._h)))
        self.n, self.m = int(n), m

    def build(self, rank_mode: int = RANK_DEGENERACY, cache_triangles: bool = False,
              rank_seed: int = 0, allocator=None) -> "Graph":
        """allocator: None (the library's own) or "torch" (PyTorch's caching allocator)
        for the index's device memory."""
        o = BuildOpts(int(rank_mode), 1 if cache_triangles else 0, int(rank_seed))
        if allocator == "torch":
            self._alloc_cbs = torch_allocator()  # kept alive as long as the graph
            o.alloc, o.free = self._alloc_cbs
        elif allocator is not None:
            raise ValueError("allocator must be None or 'torch'")
        _check(load_library().folty_build_index(self._h, ctypes.byref(o)))
        return self

    def query_noalloc(self, delta, theta=(1, 2), variant=0, universe=UNIVERSE_DST, exclude_other=False,
                      pair_u=None, pair_v=None, n_cert=None, edge_count=None, smaller_side=False) -> dict:
        """folty_run_fol_query_noalloc: the library allocates nothing; the outputs are the
        caller's int32/int32/uint32 (as int32) device tensors of equal length (the pair
        capacity) and, if given, an int32 device tensor of m entries for the per-edge counts.
        Returns n_pairs, n_certificates and the tensors cut to n_pairs."""
        q = make_query(delta, theta, variant, universe, exclude_other, True, smaller_side)
        cap = 0 if pair_u is None else int(pair_u.numel())
        ptr = lambda x: ctypes.c_void_p(x.data_ptr()) if x is not None else None
        for x in (pair_u, pair_v, n_cert, edge_count):
            if x is not None and (not x.is_cuda or x.dtype.itemsize != 4 or not x.is_contiguous()):
                raise ValueError("outputs are contiguous 4-byte device tensors")
        if pair_u is not None and not (pair_v.numel() == n_cert.numel() == cap):
            raise ValueError("pair_u, pair_v and n_cert must have the same length")
        if edge_count is not None and edge_count.numel() < self.m:
            raise ValueError("edge_count needs m entries")
        npairs, ncert = ctypes.c_int64(), ctypes.c_int64()
        _check(load_library().folty_run_fol_query_noalloc(self._h, ctypes.byref(q), ptr(pair_u), ptr(pair_v),
                                                          ptr(n_cert), cap, ptr(edge_count), ctypes.byref(npairs),
                                                          ctypes.byref(ncert)))
        k = int(npairs.value)
        return {"n_pairs": k, "n_certificates": int(ncert.value),
                "pair_u": None if pair_u is None else pair_u[:k], "pair_v": None if pair_v is None else pair_v[:k],
                "n_cert": None if n_cert is None else n_cert[:k], "edge_count": edge_count}

    def query(self, delta, theta=(1, 2), variant=0, universe=UNIVERSE_DST,
              exclude_other=False, counts=True, workspace: Workspace | None = None,
              smaller_side=False, one_pass=False) -> Result:
        """The exists-exists-forall query; smaller_side evaluates each run from the
        shorter of E_{a,b} and L2 (in-neighbour intervals), one_pass filters in one
        enumeration pass (per-item triangle slots); results are identical."""
        q = make_query(delta, theta, variant, universe, exclude_other, counts, smaller_side, one_pass)
        out = ctypes.c_void_p()
        lib = load_library()
        if workspace is None:
            _check(lib.folty_run_fol_query(self._h, ctypes.byref(q), ctypes.byref(out)))
        else:
            _check(lib.folty_run_fol_query_ws(self._h, ctypes.byref(q), workspace._h,
                                              ctypes.byref(out)))
        return Result(out)

    def vertex_query(self, delta, theta=(1, 2), inner=INNER_FORALL, inner_theta=(1, 2), variant=0,
                     universe=UNIVERSE_DST, exclude_other=False, counts=True) -> Result:
        """exists u forall_theta v in N(u) (forall_inner_theta | exists) w."""
        vq = VertexQuery()
        vq.edge = make_query(delta, inner_theta if inner == INNER_FORALL else (1, 1), variant, universe,
                             exclude_other, counts)
        vq.theta_num, vq.theta_den = to_theta(theta)
        vq.inner = int(inner)
        out = ctypes.c_void_p()
        _check(load_library().folty_run_vertex_query(self._h, ctypes.byref(vq), ctypes.byref(out)))
        return Result(out)

    def triad_query(self, delta, variant=0, triples=True, instances=True,
                    edge_instances=False, workspace: Workspace | None = None) -> Result:
        """exists u exists v exists w: solution triples and temporal triangles."""
        q = TriadQuery()
        q.delta = int(delta)
        q.variant = int(variant)
        q.flags = ((TRIAD_TRIPLES if triples else 0) | (TRIAD_INSTANCES if instances else 0)
                   | (TRIAD_EDGE_INSTANCES if edge_instances else 0))
        out = ctypes.c_void_p()
        lib = load_library()
        if workspace is None:
            _check(lib.folty_run_triad_query(self._h, ctypes.byref(q), ctypes.byref(out)))
        else:
            _check(lib.folty_run_triad_query_ws(self._h, ctypes.byref(q), workspace._h, ctypes.byref(out)))
        return Result(out)

    def query_raw(self, q: Query) -> Result:
        out = ctypes.c_void_p()
        _check(load_library().folty_run_fol_query(self._h, ctypes.byref(q), ctypes.byref(out)))
        return Result(out)

    def batch(self, queries) -> list:
        qs = (Query * len(queries))(*[q if isinstance(q, Query) else make_query(**q) for q in queries])
        outs = (ctypes.c_void_p * len(queries))()
        _check(load_library().folty_run_batch(self._h, qs, len(queries), outs))
        return [Result(ctypes.c_void_p(o)) for o in outs]

    def stats(self) -> dict:
        st = Stats()
        _check(load_library().folty_graph_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def vertex_array(self, what: int) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.int32)
        _check(load_library().folty_graph_vertex_array(self._h, int(what),
                                                       ctypes.c_void_p(out.ctypes.data)))
        return out

    def degrees(self):
        return self.vertex_array(0)

    def core_numbers(self):
        return self.vertex_array(1)

    def ranks(self):
        return self.vertex_array(2)

    def out_degrees(self):
        return self.vertex_array(3)

    def device_bytes(self) -> int:
        b = ctypes.c_int64()
        _check(load_library().folty_graph_device_bytes(self._h, ctypes.byref(b)))
        return b.value

    def close(self):
        if getattr(self, "_h", None):
            load_library().folty_graph_free(self._h)
            self._h = None
        self._inputs = None  # borrowed tensors: the library no longer reads them

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_multi(graphs, queries) -> list:
    """One query per graph, all graphs in one call."""
    n = len(graphs)
    gs = (ctypes.c_void_p * n)(*[g._h.value for g in graphs])
    qs = (Query * n)(*[q if isinstance(q, Query) else make_query(**q) for q in queries])
    outs = (ctypes.c_void_p * n)()
    _check(load_library().folty_run_multi(gs, qs, n, outs))
    return [Result(ctypes.c_void_p(o)) for o in outs]


class Plan:
    """A fixed batch of queries over resident graphs, run as one captured launch
    sequence.  `queries` is a list of (graph_index, query) where query is a dict
    of make_query's arguments or a Query."""

    def __init__(self, graphs, queries):
        self.graphs = list(graphs)  # keep the graphs alive as long as the plan
        n = len(queries)
        gs = (ctypes.c_void_p * len(self.graphs))(*[g._h.value for g in self.graphs])
        qs = (Query * max(1, n))(*[q if isinstance(q, Query) else make_query(**q) for _, q in queries])
        qg = (ctypes.c_int32 * max(1, n))(*[int(gi) for gi, _ in queries])
        self.n = n
        self._h = ctypes.c_void_p()
        _check(load_library().folty_plan_create(gs, len(self.graphs), qs, qg, n, ctypes.byref(self._h)))

    def run(self) -> list:
        outs = (ctypes.c_void_p * max(1, self.n))()
        _check(load_library().folty_plan_run(self._h, outs))
        return [Result(ctypes.c_void_p(outs[i])) for i in range(self.n)]

    def info(self) -> dict:
        info = PlanInfo()
        _check(load_library().folty_plan_get_info(self._h, ctypes.byref(info)))
        return info.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            load_library().folty_plan_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching query server over resident graphs (thread-safe)."""

    def __init__(self, workers: int = 4, max_batch: int = 16, hbm_budget_bytes: int = 0):
        o = ServerOpts(int(workers), int(max_batch), int(hbm_budget_bytes))
        self._h = ctypes.c_void_p()
        _check(load_library().folty_server_create(ctypes.byref(o), ctypes.byref(self._h)))

    def submit(self, graph: "Graph", **query) -> int:
        q = query.pop("query", None) or make_query(**query)
        t = ctypes.c_int64()
        _check(load_library().folty_server_submit(self._h, graph._h, ctypes.byref(q), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """The result, or None while the request is not done."""
        out = ctypes.c_void_p()
        rc = load_library().folty_server_poll(self._h, int(ticket), ctypes.byref(out))
        if rc == EBUSY:
            return None
        _check(rc)
        return Result(out)

    def wait(self, ticket: int) -> Result:
        out = ctypes.c_void_p()
        _check(load_library().folty_server_wait(self._h, int(ticket), ctypes.byref(out)))
        return Result(out)

    def info(self) -> dict:
        i = ServerInfo()
        _check(load_library().folty_server_get_info(self._h, ctypes.byref(i)))
        return i.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            load_library().folty_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def release_cached_memory() -> int:
    """Hand the library's cached device blocks and pinned host blocks back to the
    driver; returns bytes."""
    b = ctypes.c_int64()
    _check(load_library().folty_release_cached_memory(ctypes.byref(b)))
    return b.value


def version() -> str:
    return load_library().folty_version().decode()
