"""Python binding of libged (include/ged.h): argument marshalling only.

Every step of the search runs in the HIP kernels of libged.so; this module
only converts numpy / torch arguments to the C ABI.  torch provides device
memory and streams.  If libged.so is missing the import of this module
fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np
import torch  # noqa: F401  -- load torch's HIP runtime before libged binds to it

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libged.so")

GED_OK, GED_EINVAL, GED_ENOMEM, GED_EUNSUPPORTED, GED_EDEVICE, GED_EBUSY, GED_ETIMEOUT, GED_ECANCELED = range(8)
MAX_VERTICES = 1024           # databases, the single-pair search, edit paths
MAX_VERTICES_BATCH = 512      # batched plans, the per-pair path, serving
MAX_K = 1024
MAX_K_WIDE = 1 << 21
MAX_EDGE_LABELS = 16


class GedError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_name(status) if _lib else status}: {message}")
        self.status = status


SCHED_AUTO, SCHED_BLOCK = 0, 1
LAST_SELECT, LAST_COMPLETE = 0, 1
METHOD_TREE, METHOD_BIPARTITE = 0, 1
BIP_MAX_ORDER, BIP_MAX_K = 256, 256
DB_DIRECTED = 1                 # ged_db_create_ex flag: edge k is the arc eu[k] -> ev[k]
DIRECTED_MAX_ORDER = 256
PLAN_PAIR_STATUS = 1            # ged_plan_options.flags: set unsearchable pairs aside with a status each
NOALLOC_SCRATCH_BYTES = 64 << 20


class PlanOptions(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("groups_per_cu", ctypes.c_int32), ("last_level", ctypes.c_int32),
                ("method", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Costs(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in ("vsub", "vdel", "vins", "esub", "edel", "eins")]


class GraphStruct(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("vlabel", ctypes.c_void_p),
                ("eu", ctypes.c_void_p), ("ev", ctypes.c_void_p), ("elabel", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("costs", Costs), ("hbm_budget", ctypes.c_int64),
                ("max_inflight", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("queue_capacity", ctypes.c_int32), ("method", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("submitted", "completed", "rejected_busy", "launches", "queued",
                                              "inflight", "inflight_peak", "batch_peak", "device_bytes")]


# Layout of ged_graph: int32 n, m; then four pointers (x86-64: 40 bytes).
GRAPH_DTYPE = np.dtype([("n", "<i4"), ("m", "<i4"), ("vlabel", "<u8"), ("eu", "<u8"),
                        ("ev", "<u8"), ("elabel", "<u8")])

_lib = None

EXPORTS = (
    "ged_abi_version", "ged_last_error", "ged_status_name",
    "ged_db_create", "ged_db_destroy", "ged_db_count", "ged_db_device_bytes", "ged_db_order",
    "ged_db_create_ex", "ged_db_flags",
    "ged_plan_create", "ged_plan_map_size", "ged_plan_run", "ged_plan_run_perpair",
    "ged_plan_destroy", "ged_kbest", "ged_kbest_perpair",
    "ged_plan_set_timing", "ged_plan_kernel_ms", "ged_plan_kernel_launches",
    "ged_plan_create_ex", "ged_plan_bin_count", "ged_plan_bin_info",
    "ged_plan_capture", "ged_plan_replay", "ged_plan_tune",
    "ged_server_create", "ged_server_submit", "ged_server_poll", "ged_server_wait",
    "ged_server_stats_get", "ged_server_destroy", "ged_server_submit_batch", "ged_server_collect",
    "ged_wide_create", "ged_wide_create_ex", "ged_wide_bytes", "ged_wide_run", "ged_wide_destroy",
    "ged_edit_path_capacity", "ged_edit_path",
    "ged_plan_run_ex", "ged_kbest_ex", "ged_map_offsets", "ged_kbest_noalloc", "ged_server_submit_id",
)


def load(path: str = LIB_PATH):
    """Load libged.so and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() "
                          f"(or python paper_2605_00830_amd/build.py)")
    lib = ctypes.CDLL(path)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "ged_abi_version": ([], i32),
        "ged_last_error": ([], ctypes.c_char_p),
        "ged_status_name": ([i32], ctypes.c_char_p),
        "ged_db_create": ([P, i64, P], i32),
        "ged_db_create_ex": ([P, i64, ctypes.c_uint32, P], i32),
        "ged_db_flags": ([P, P], i32),
        "ged_db_destroy": ([P], i32),
        "ged_db_count": ([P, P], i32),
        "ged_db_device_bytes": ([P, P], i32),
        "ged_db_order": ([P, i64, P], i32),
        "ged_plan_create": ([P, P, i64, i32, P], i32),
        "ged_plan_map_size": ([P, P], i32),
        "ged_plan_run": ([P, Costs, P, P, P, P], i32),
        "ged_plan_run_perpair": ([P, Costs, P, P, P, P], i32),
        "ged_plan_destroy": ([P], i32),
        "ged_kbest": ([P, P, i64, Costs, i32, P, P, P], i32),
        "ged_kbest_perpair": ([P, P, i64, Costs, i32, P, P, P], i32),
        "ged_plan_set_timing": ([P, i32], i32),
        "ged_plan_kernel_ms": ([P, P], i32),
        "ged_plan_kernel_launches": ([P, P], i32),
        "ged_plan_create_ex": ([P, P, i64, i32, P, P], i32),
        "ged_plan_bin_count": ([P, P], i32),
        "ged_plan_bin_info": ([P, i32, P, P, P, P], i32),
        "ged_plan_capture": ([P, Costs, P, P, P, P], i32),
        "ged_plan_replay": ([P, P], i32),
        "ged_plan_tune": ([P, Costs, P, P, P, ctypes.c_char_p, P], i32),
        "ged_server_create": ([P, P, P], i32),
        "ged_server_submit": ([P, P, i64, P], i32),
        "ged_server_poll": ([P, ctypes.c_uint64, P, P, i32, P, P], i32),
        "ged_server_wait": ([P, ctypes.c_uint64, i64, P, P, i32, P, P], i32),
        "ged_server_submit_batch": ([P, P, P, i64, P, P], i32),
        "ged_server_collect": ([P, i64, i64, P, P, P, P, i64, P], i32),
        "ged_server_stats_get": ([P, P], i32),
        "ged_server_destroy": ([P], i32),
        "ged_wide_create": ([P, i64, i64, i32, P], i32),
        "ged_wide_create_ex": ([P, i64, i64, i32, P, P], i32),
        "ged_wide_bytes": ([P, P], i32),
        "ged_wide_run": ([P, Costs, P, P, P, P], i32),
        "ged_wide_destroy": ([P], i32),
        "ged_edit_path_capacity": ([P, P, i64, P], i32),
        "ged_edit_path": ([P, P, i64, Costs, P, P, P, P], i32),
        "ged_plan_run_ex": ([P, Costs, P, P, P, P, P], i32),
        "ged_kbest_ex": ([P, P, i64, Costs, i32, P, P, P, P, P, P], i32),
        "ged_map_offsets": ([P, P, i64, P, P], i32),
        "ged_kbest_noalloc": ([P, P, i64, Costs, i32, P, P, P], i32),
        "ged_server_submit_id": ([P, i64, i64, P], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def status_name(status: int) -> str:
    return load().ged_status_name(int(status)).decode()


def _check(status: int):
    if status != GED_OK:
        msg = load().ged_last_error().decode(errors="replace")
        raise GedError(status, msg)


def _costs(c: Sequence[int]) -> Costs:
    if len(c) != 6:
        raise ValueError("costs are (vsub, vdel, vins, esub, edel, eins)")
    return Costs(*[int(x) for x in c])


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class Database:
    """A device-resident graph database (ged_db_create_ex); `graphs` is a synth.GraphSet.
    directed: every graph is directed, edge k being the arc eu[k] -> ev[k]."""

    def __init__(self, graphs, directed: bool = False):
        lib = load()
        torch.cuda.init()
        count = len(graphs)
        vl = np.ascontiguousarray(graphs.vlabel, dtype=np.int32)
        eu = np.ascontiguousarray(graphs.eu, dtype=np.int32)
        ev = np.ascontiguousarray(graphs.ev, dtype=np.int32)
        el = None if graphs.elabel is None else np.ascontiguousarray(graphs.elabel, dtype=np.int32)
        recs = np.zeros(max(count, 1), dtype=GRAPH_DTYPE)
        recs["n"][:count] = graphs.n
        recs["m"][:count] = graphs.m
        voff = np.asarray(graphs.voff, dtype=np.uint64)[:count]
        eoff = np.asarray(graphs.eoff, dtype=np.uint64)[:count]
        recs["vlabel"][:count] = np.uint64(vl.ctypes.data) + voff * np.uint64(4)
        recs["eu"][:count] = np.uint64(eu.ctypes.data) + eoff * np.uint64(4)
        recs["ev"][:count] = np.uint64(ev.ctypes.data) + eoff * np.uint64(4)
        if el is not None:
            recs["elabel"][:count] = np.uint64(el.ctypes.data) + eoff * np.uint64(4)
        handle = ctypes.c_void_p()
        _check(lib.ged_db_create_ex(recs.ctypes.data, count, DB_DIRECTED if directed else 0,
                                    ctypes.byref(handle)))
        self._h = handle
        self.directed = bool(directed)
        self.count = count
        self.n = np.asarray(graphs.n, dtype=np.int32).copy()

    @property
    def handle(self):
        if self._h is None:
            raise GedError(GED_EINVAL, "database is closed")
        return self._h

    def device_bytes(self) -> int:
        out = ctypes.c_int64()
        _check(load().ged_db_device_bytes(self.handle, ctypes.byref(out)))
        return int(out.value)

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().ged_db_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _pairs_array(pairs) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))


class Plan:
    """A reusable batched launch plan (ged_plan_create)."""

    def __init__(self, db: Database, pairs, K: int, schedule: int = SCHED_AUTO, groups_per_cu: int = 0,
                 last_level: int = LAST_SELECT, method: int = METHOD_TREE, flags: int = 0):
        lib = load()
        self.db = db
        self.pairs = _pairs_array(pairs)
        self.K = int(K)
        handle = ctypes.c_void_p()
        opt = PlanOptions(int(schedule), int(groups_per_cu), int(last_level), int(method), int(flags))
        _check(lib.ged_plan_create_ex(db.handle, self.pairs.ctypes.data, len(self.pairs), self.K,
                                      ctypes.byref(opt), ctypes.byref(handle)))
        self._h = handle
        size = ctypes.c_int64()
        _check(lib.ged_plan_map_size(self._h, ctypes.byref(size)))
        self.map_size = int(size.value)
        # where each pair's mapping starts (ids out of range take no entries)
        src = self.pairs[:, 0] if len(self.pairs) else np.zeros(0, np.int64)
        ok = (src >= 0) & (src < db.count)
        n_src = np.where(ok, db.n[np.where(ok, src, 0)] if db.count else 0, 0).astype(np.int64)
        self.offsets = np.zeros(len(self.pairs), dtype=np.int64)
        if len(self.pairs) > 1:
            np.cumsum(n_src[:-1], out=self.offsets[1:])

    def outputs(self, device="cuda", with_cand: bool = False):
        dist = torch.empty(max(len(self.pairs), 1), dtype=torch.int32, device=device)
        maps = torch.empty(max(self.map_size, 1), dtype=torch.int32, device=device)
        cand = torch.empty(max(len(self.pairs), 1), dtype=torch.int64, device=device) if with_cand else None
        return dist, maps, cand

    def _check_outputs(self, dist, maps, cand):
        for t, dt in ((dist, torch.int32), (maps, torch.int32)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError("outputs must be contiguous int32 CUDA tensors")
        if dist.numel() < len(self.pairs) or maps.numel() < self.map_size:
            raise ValueError("output tensors are too small")
        if cand is not None and (cand.dtype != torch.int64 or not cand.is_cuda or cand.numel() < len(self.pairs)):
            raise ValueError("cand must be an int64 CUDA tensor of npairs entries")

    def run(self, costs, dist: torch.Tensor, maps: torch.Tensor, cand: Optional[torch.Tensor] = None,
            stream=None, perpair: bool = False, status: Optional[torch.Tensor] = None):
        """ged_plan_run (ged_plan_run_ex with `status`, an int32 tensor of npairs
        entries for the per-pair statuses; ged_plan_run_perpair with perpair)."""
        lib = load()
        self._check_outputs(dist, maps, cand)
        cp = None if cand is None else cand.data_ptr()
        if status is not None:
            if perpair:
                raise ValueError("the per-pair path reports no statuses")
            if status.dtype != torch.int32 or not status.is_cuda or status.numel() < len(self.pairs):
                raise ValueError("status must be an int32 CUDA tensor of npairs entries")
            _check(lib.ged_plan_run_ex(self._h, _costs(costs), dist.data_ptr(), maps.data_ptr(), cp,
                                       status.data_ptr(), _stream_handle(stream)))
            return
        fn = lib.ged_plan_run_perpair if perpair else lib.ged_plan_run
        _check(fn(self._h, _costs(costs), dist.data_ptr(), maps.data_ptr(), cp, _stream_handle(stream)))

    def set_timing(self, enable: bool = True):
        _check(load().ged_plan_set_timing(self._h, 1 if enable else 0))

    def kernel_ms(self) -> float:
        """Elapsed ms between the events around the last run's search kernels
        (the stream must have been synchronized)."""
        out = ctypes.c_float()
        _check(load().ged_plan_kernel_ms(self._h, ctypes.byref(out)))
        return float(out.value)

    def capture(self, costs, dist: torch.Tensor, maps: torch.Tensor, cand: Optional[torch.Tensor] = None,
                stream=None):
        """Record one run into a HIP graph owned by the plan (stream must not be the null stream)."""
        self._check_outputs(dist, maps, cand)
        _check(load().ged_plan_capture(self._h, _costs(costs), dist.data_ptr(), maps.data_ptr(),
                                       None if cand is None else cand.data_ptr(), _stream_handle(stream)))

    def replay(self, stream=None):
        _check(load().ged_plan_replay(self._h, _stream_handle(stream)))

    def tune(self, costs, dist: torch.Tensor, maps: torch.Tensor, stream=None,
             cache_path: Optional[str] = None) -> int:
        """Pick each bin's fastest schedule (see ged_plan_tune); returns the bins timed."""
        self._check_outputs(dist, maps, None)
        timed = ctypes.c_int32(0)
        _check(load().ged_plan_tune(self._h, _costs(costs), dist.data_ptr(), maps.data_ptr(),
                                    _stream_handle(stream),
                                    None if cache_path is None else cache_path.encode(),
                                    ctypes.byref(timed)))
        return int(timed.value)

    def bins(self):
        """[(kernel name, pairs, grid, words)] for each size bin, in launch order."""
        lib = load()
        cnt = ctypes.c_int32()
        _check(lib.ged_plan_bin_count(self._h, ctypes.byref(cnt)))
        out = []
        for k in range(cnt.value):
            kern, npairs, grid, words = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
            _check(lib.ged_plan_bin_info(self._h, k, ctypes.byref(kern), ctypes.byref(npairs),
                                         ctypes.byref(grid), ctypes.byref(words)))
            if kern.value == 0:
                name = "kb_wave_kernel" if words.value == 1 else "kb_wave2_kernel"
            elif kern.value == 2:
                name = "kb_bip_kernel"
            else:
                name = "kb_block_kernel"
            out.append((name, int(npairs.value), int(grid.value), int(words.value)))
        return out

    def kernel_launches(self) -> int:
        out = ctypes.c_int64()
        _check(load().ged_plan_kernel_launches(self._h, ctypes.byref(out)))
        return int(out.value)

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().ged_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Result:
    dist: np.ndarray      # int32 [P]
    maps: np.ndarray      # int32 [sum n(src)], -1 = deleted
    offsets: np.ndarray   # int64 [P]
    cand: Optional[np.ndarray] = None  # int64 [P] children evaluated (bipartite: assignment problems solved)

    def mapping(self, p: int, n1: int) -> np.ndarray:
        o = int(self.offsets[p])
        return self.maps[o:o + n1]


def kbest(db: Database, pairs, costs, K: int, perpair: bool = False, with_cand: bool = False,
          stream=None, schedule: int = SCHED_AUTO, groups_per_cu: int = 0, last_level: int = LAST_SELECT,
          method: int = METHOD_TREE) -> Result:
    """K-Best GED of every (src, dst) pair; synchronizes and returns host arrays."""
    plan = Plan(db, pairs, K, schedule=schedule, groups_per_cu=groups_per_cu, last_level=last_level, method=method)
    try:
        dist, maps, cand = plan.outputs(with_cand=with_cand)
        plan.run(costs, dist, maps, cand, stream=stream, perpair=perpair)
        (stream or torch.cuda.current_stream()).synchronize()
        n = len(plan.pairs)
        return Result(dist[:n].cpu().numpy(), maps[:plan.map_size].cpu().numpy(), plan.offsets.copy(),
                      None if cand is None else cand[:n].cpu().numpy())
    finally:
        plan.close()


def kbest_ex(db: Database, pairs, costs, K: int, last_level: int = LAST_SELECT, method: int = METHOD_TREE,
             flags: int = PLAN_PAIR_STATUS, stream=None):
    """ged_kbest_ex: (Result with cand, status int32 [P]); synchronizes."""
    lib = load()
    pairs = _pairs_array(pairs)
    P = len(pairs)
    opt = PlanOptions(SCHED_AUTO, 0, int(last_level), int(method), int(flags))
    # output sizes from the same layout the library uses
    src = pairs[:, 0] if P else np.zeros(0, np.int64)
    ok = (src >= 0) & (src < db.count)
    n_src = np.where(ok, db.n[np.where(ok, src, 0)] if db.count else 0, 0).astype(np.int64)
    off = np.zeros(P, dtype=np.int64)
    if P > 1:
        np.cumsum(n_src[:-1], out=off[1:])
    total = int(n_src.sum())
    dist = torch.empty(max(P, 1), dtype=torch.int32, device="cuda")
    maps = torch.empty(max(total, 1), dtype=torch.int32, device="cuda")
    cand = torch.empty(max(P, 1), dtype=torch.int64, device="cuda")
    status = torch.empty(max(P, 1), dtype=torch.int32, device="cuda")
    _check(lib.ged_kbest_ex(db.handle, pairs.ctypes.data, P, _costs(costs), int(K), ctypes.byref(opt),
                            dist.data_ptr(), maps.data_ptr(), cand.data_ptr(), status.data_ptr(),
                            _stream_handle(stream)))
    return (Result(dist[:P].cpu().numpy(), maps[:total].cpu().numpy(), off, cand[:P].cpu().numpy()),
            status[:P].cpu().numpy())


def map_offsets(db: Database, d_pairs: torch.Tensor, stream=None) -> torch.Tensor:
    """ged_map_offsets on device pairs (int64 tensor [P, 2]): int64 tensor [P + 1]."""
    if d_pairs.dtype != torch.int64 or not d_pairs.is_cuda or not d_pairs.is_contiguous():
        raise ValueError("d_pairs must be a contiguous int64 CUDA tensor of shape [P, 2]")
    P = d_pairs.numel() // 2
    off = torch.empty(P + 1, dtype=torch.int64, device=d_pairs.device)
    _check(load().ged_map_offsets(db.handle, d_pairs.data_ptr() if P else None, P, off.data_ptr(),
                                  _stream_handle(stream)))
    return off


def kbest_noalloc(db: Database, pairs, costs, K: int, dist: torch.Tensor, maps: torch.Tensor, stream=None):
    """ged_kbest_noalloc into caller-owned outputs (int32 CUDA tensors of P and sum n(src)
    entries); synchronizes the stream."""
    pairs = _pairs_array(pairs)
    for t in (dist, maps):
        if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("outputs must be contiguous int32 CUDA tensors")
    _check(load().ged_kbest_noalloc(db.handle, pairs.ctypes.data if len(pairs) else None, len(pairs),
                                    _costs(costs), int(K), dist.data_ptr(), maps.data_ptr(),
                                    _stream_handle(stream)))


class Wide:
    """Single-pair search at large K with the whole device (ged_wide_*)."""

    def __init__(self, db: Database, src: int, dst: int, K: int, last_level: int = LAST_SELECT):
        lib = load()
        self.db = db
        self.src, self.dst, self.K = int(src), int(dst), int(K)
        handle = ctypes.c_void_p()
        opt = PlanOptions(SCHED_AUTO, 0, int(last_level), METHOD_TREE, 0)
        _check(lib.ged_wide_create_ex(db.handle, self.src, self.dst, self.K, ctypes.byref(opt), ctypes.byref(handle)))
        self._h = handle
        self.n1 = int(db.n[self.src])
        size = ctypes.c_int64()
        _check(lib.ged_wide_bytes(self._h, ctypes.byref(size)))
        self.bytes = int(size.value)

    def outputs(self, device="cuda"):
        dist = torch.empty(1, dtype=torch.int32, device=device)
        maps = torch.empty(max(self.n1, 1), dtype=torch.int32, device=device)
        cand = torch.empty(1, dtype=torch.int64, device=device)
        return dist, maps, cand

    def run(self, costs, dist: torch.Tensor, maps: torch.Tensor, cand: Optional[torch.Tensor] = None, stream=None):
        for t, dt, n in ((dist, torch.int32, 1), (maps, torch.int32, self.n1)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous() or t.numel() < n:
                raise ValueError("outputs must be contiguous int32 CUDA tensors of 1 and n1 entries")
        if cand is not None and (cand.dtype != torch.int64 or not cand.is_cuda):
            raise ValueError("cand must be an int64 CUDA tensor")
        _check(load().ged_wide_run(self._h, _costs(costs), dist.data_ptr(), maps.data_ptr(),
                                   None if cand is None else cand.data_ptr(), _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().ged_wide_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kbest_wide(db: Database, src: int, dst: int, costs, K: int, stream=None, last_level: int = LAST_SELECT):
    """(dist, mapping, children evaluated) of one pair by the large-K search; synchronizes."""
    w = Wide(db, src, dst, K, last_level=last_level)
    try:
        dist, maps, cand = w.outputs()
        w.run(costs, dist, maps, cand, stream=stream)
        (stream or torch.cuda.current_stream()).synchronize()
        return int(dist.item()), maps[:w.n1].cpu().numpy(), int(cand.item())
    finally:
        w.close()


def _graph_struct(g, keep: list) -> GraphStruct:
    arrs = []
    for a in (g.vlabel, g.eu, g.ev, getattr(g, "elabel", None)):
        arrs.append(None if a is None else np.ascontiguousarray(a, dtype=np.int32))
    keep.extend(arrs)
    ptr = [None if a is None or a.size == 0 else a.ctypes.data for a in arrs]
    return GraphStruct(int(g.n), int(arrs[1].shape[0]), ptr[0], ptr[1], ptr[2], ptr[3])


class Server:
    """The serving loop (ged_server_*): submit (query graph, target id), poll or wait."""

    def __init__(self, db: Database, K: int, costs, hbm_budget: int = 0, max_inflight: int = 0,
                 max_batch: int = 0, streams: int = 0, queue_capacity: int = 0, method: int = METHOD_TREE):
        lib = load()
        self.db = db
        cfg = ServerConfig(int(K), _costs(costs), int(hbm_budget), int(max_inflight), int(max_batch),
                           int(streams), int(queue_capacity), int(method))
        handle = ctypes.c_void_p()
        _check(lib.ged_server_create(db.handle, ctypes.byref(cfg), ctypes.byref(handle)))
        self._h = handle

    def submit(self, query, target_id: int) -> int:
        """Queue one query; raises GedError (status GED_EBUSY when the queue is full)."""
        keep: list = []
        gs = _graph_struct(query, keep)
        t = ctypes.c_uint64()
        _check(load().ged_server_submit(self._h, ctypes.byref(gs), int(target_id), ctypes.byref(t)))
        return int(t.value)

    def submit_id(self, query_id: int, target_id: int) -> int:
        """Queue database graph `query_id` against `target_id` (ged_server_submit_id)."""
        t = ctypes.c_uint64()
        _check(load().ged_server_submit_id(self._h, int(query_id), int(target_id), ctypes.byref(t)))
        return int(t.value)

    def _result(self, fn, *args):
        # the mapping and the times land in buffers of this call's own: wait and
        # poll may run on several client threads at once
        d, n1 = ctypes.c_int32(), ctypes.c_int32()
        times = (ctypes.c_int64 * 2)()
        buf = np.empty(MAX_VERTICES_BATCH, dtype=np.int32)
        st = fn(self._h, *args, ctypes.byref(d), buf.ctypes.data, MAX_VERTICES_BATCH, ctypes.byref(n1), times)
        return st, int(d.value), buf[: n1.value].copy(), (int(times[0]), int(times[1]))

    def poll(self, ticket: int, with_times: bool = False):
        """(dist, mapping) when finished, None while it runs; with_times adds the
        (submission, completion) times of this query (monotonic clock, ns)."""
        st, d, m, t = self._result(load().ged_server_poll, ctypes.c_uint64(ticket))
        if st == GED_EBUSY:
            return None
        _check(st)
        return (d, m, t) if with_times else (d, m)

    def wait(self, ticket: int, timeout_us: int = -1, with_times: bool = False):
        st, d, m, t = self._result(load().ged_server_wait, ctypes.c_uint64(ticket), int(timeout_us))
        _check(st)
        return (d, m, t) if with_times else (d, m)

    def submit_batch(self, recs: np.ndarray, targets: np.ndarray) -> np.ndarray:
        """Submit ged_graph records (GRAPH_DTYPE array, see pack_queries) in order; returns
        the tickets of those queued (fewer than given when the queue filled up)."""
        recs = np.ascontiguousarray(recs)
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        tickets = np.zeros(max(len(recs), 1), dtype=np.uint64)
        acc = ctypes.c_int64()
        st = load().ged_server_submit_batch(self._h, recs.ctypes.data, targets.ctypes.data, len(recs),
                                            tickets.ctypes.data, ctypes.byref(acc))
        if st not in (GED_OK, GED_EBUSY):
            _check(st)
        return tickets[: acc.value]

    def collect(self, max_count: int = 4096, timeout_us: int = -1, with_maps: bool = False):
        """(tickets, dist, times_ns [k,2], maps or None) of finished queries, or None on timeout."""
        lib = load()
        tickets = np.zeros(max_count, np.uint64)
        dist = np.zeros(max_count, np.int32)
        times = np.zeros((max_count, 2), np.int64)
        maps = np.zeros(max_count * 64, np.int32) if with_maps else None
        cnt = ctypes.c_int64()
        st = lib.ged_server_collect(self._h, int(timeout_us), int(max_count), tickets.ctypes.data,
                                    dist.ctypes.data, times.ctypes.data,
                                    None if maps is None else maps.ctypes.data,
                                    0 if maps is None else maps.shape[0], ctypes.byref(cnt))
        if st == GED_ETIMEOUT:
            return None
        _check(st)
        n = int(cnt.value)
        return tickets[:n], dist[:n], times[:n], maps

    def stats(self) -> dict:
        out = ServerStats()
        _check(load().ged_server_stats_get(self._h, ctypes.byref(out)))
        return {f: int(getattr(out, f)) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().ged_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pack_queries(graphs) -> Tuple[np.ndarray, list]:
    """ged_graph records (GRAPH_DTYPE) for a GraphSet's graphs; returns (records, arrays to keep alive)."""
    vl = np.ascontiguousarray(graphs.vlabel, dtype=np.int32)
    eu = np.ascontiguousarray(graphs.eu, dtype=np.int32)
    ev = np.ascontiguousarray(graphs.ev, dtype=np.int32)
    el = None if graphs.elabel is None else np.ascontiguousarray(graphs.elabel, dtype=np.int32)
    count = len(graphs)
    recs = np.zeros(count, dtype=GRAPH_DTYPE)
    recs["n"] = graphs.n
    recs["m"] = graphs.m
    voff = np.asarray(graphs.voff, dtype=np.uint64)[:count]
    eoff = np.asarray(graphs.eoff, dtype=np.uint64)[:count]
    recs["vlabel"] = np.uint64(vl.ctypes.data) + voff * np.uint64(4)
    recs["eu"] = np.uint64(eu.ctypes.data) + eoff * np.uint64(4)
    recs["ev"] = np.uint64(ev.ctypes.data) + eoff * np.uint64(4)
    if el is not None:
        recs["elabel"] = np.uint64(el.ctypes.data) + eoff * np.uint64(4)
    return recs, [vl, eu, ev, el]


# ------------------------------------------------------------------ edit paths

OP_VSUB, OP_VDEL, OP_VINS, OP_ESUB, OP_EDEL, OP_EINS = range(6)
OP_NAMES = ("vsub", "vdel", "vins", "esub", "edel", "eins")


def edit_path(db: Database, pairs, costs, maps: torch.Tensor, stream=None):
    """Explicit edit operations of each pair's mapping (ged_edit_path).

    maps: the device mappings in the searches' layout (Plan.outputs / Result order).
    Returns (ops int32 [total, 6] as (kind, a, b, c, d, cost), offsets int64 [P + 1],
    counts int32 [P]); pair p's operations are ops[offsets[p] : offsets[p] + counts[p]].
    """
    lib = load()
    pairs = _pairs_array(pairs)
    P = len(pairs)
    off = np.zeros(P + 1, dtype=np.int64)
    _check(lib.ged_edit_path_capacity(db.handle, pairs.ctypes.data, P, off.ctypes.data))
    if maps.dtype != torch.int32 or not maps.is_cuda or not maps.is_contiguous():
        raise ValueError("maps must be a contiguous int32 CUDA tensor")
    ops = torch.empty(max(int(off[-1]), 1) * 6, dtype=torch.int32, device=maps.device)
    count = torch.empty(max(P, 1), dtype=torch.int32, device=maps.device)
    _check(lib.ged_edit_path(db.handle, pairs.ctypes.data, P, _costs(costs), maps.data_ptr(), ops.data_ptr(),
                             count.data_ptr(), _stream_handle(stream)))
    return ops.view(-1, 6)[: int(off[-1])].cpu().numpy(), off, count[:P].cpu().numpy()
