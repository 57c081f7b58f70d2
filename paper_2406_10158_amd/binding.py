"""Python binding of the C-ABI in include/cc.h (argument marshalling only).

Every function here has the name of the C entry point it calls and does no
transaction work itself: all of it runs in libcc.so's HIP kernels.  Importing
this module loads libcc.so and raises ImportError if it has not been built
(``python -m paper_2406_10158_amd.build``) -- there is no fallback path.

Arrays: host arguments are numpy arrays; device arguments are objects with a
``data_ptr()`` method (torch tensors on the context's GPU).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcc.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2406_10158_amd.build`")
lib = ctypes.CDLL(_LIB_PATH)

# ---- constants (mirror include/cc.h) ---------------------------------------
CC_OK = 0
CC_E_INVAL, CC_E_RANGE, CC_E_DUPROW, CC_E_NOMEM, CC_E_TS_OVERFLOW = -1, -2, -3, -4, -5
CC_E_LIVELOCK, CC_E_HIP, CC_E_NODEV, CC_E_STATE, CC_E_NOBATCH = -6, -7, -8, -9, -10
CC_OCC, CC_2PL_NW, CC_TO, CC_MVCC, CC_TICTOC, CC_GACCO, CC_2PL_WD, CC_GPUTX = 0, 1, 2, 3, 4, 5, 6, 7
SCHEMES = {"occ": CC_OCC, "2pl_nw": CC_2PL_NW, "to": CC_TO, "mvcc": CC_MVCC, "tictoc": CC_TICTOC,
           "gacco": CC_GACCO, "2pl_wd": CC_2PL_WD, "gputx": CC_GPUTX}
CC_READ, CC_ADD, CC_COND_ADD, CC_WRITE_SLOT = 0, 1, 2, 3
CC_PENDING, CC_COMMITTED = 0, 1
CC_MODE_PLAIN, CC_MODE_EPOCH, CC_MODE_SERVE = 0, 1, 2
CC_SERVE_BYTES_PER_OP = 32
CC_RUN_STRICT_FENCES = 0x1
CC_RUN_EAGER_INSTALL = 0x2
CC_RUN_WAIT_UNLOCK = 0x4
CC_RUN_PRECHECK = 0x8
CC_RUN_NO_PRECHECK = 0x10
CC_RUN_INDEX_TREE = 0x20
CC_RUN_LATCH = 0x40
CC_RUN_SHARED_READS = 0x80
CC_RUN_HOT_LAST = 0x100
CC_RUN_NO_HOT_LAST = 0x200
CC_RUN_WAIT_BLOCKER = 0x400
CC_RUN_HOT_ENGINE = 0x800
CC_RUN_NO_HOT_ENGINE = 0x1000
STAT_NAMES = ["committed", "attempts", "abort_lock", "abort_valid", "kernel_ns", "run_ns", "tickets",
              "max_attempts", "lat_p50_ns", "lat_p99_ns", "epochs", "passes", "deferred", "grid",
              "t_useful_ns", "t_abort_ns", "t_wait_ns", "gave_up", "admit_waits",
              "occ_r1_ns", "occ_r2_ns", "occ_r3_ns", "occ_r4_ns", "prep_ns", "index_ns", "wd_waits", "ksets",
              "packed_state", "hot_acq", "hot_failed", "hot_hold_ns", "hot_writes", "blocked_waits",
              "version_slots", "version_misses", "engine_txns", "engine_rows", "engine_ns", "engine_waits"]
CC_N_STATS = 40
CC_STATIC_MAX_TXNS = 1 << 18
CC_STATIC_MAX_OPS = 1 << 20

OP_DTYPE = np.dtype([("row", "<u4"), ("table", "<u2"), ("field", "u1"), ("kind", "u1"), ("arg", "<i8")])
TXN_DTYPE = np.dtype([("first_op", "<u8"), ("n_ops", "<u4"), ("reserved", "<u4")])
OUTCOME_DTYPE = np.dtype([("status", "<u4"), ("attempts", "<u4"), ("serial_hi", "<u8"), ("serial_lo", "<u8"),
                          ("commit_ns", "<i8")])
assert OP_DTYPE.itemsize == 16 and TXN_DTYPE.itemsize == 16 and OUTCOME_DTYPE.itemsize == 32


class cc_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("flags", ctypes.c_uint32), ("stream", ctypes.c_void_p)]


class cc_run_params(ctypes.Structure):
    _fields_ = [("lanes_per_txn", ctypes.c_uint32), ("waves_per_wg", ctypes.c_uint32), ("grid", ctypes.c_uint32),
                ("mode", ctypes.c_uint32), ("max_attempts", ctypes.c_uint64), ("max_epochs", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("backoff_ns", ctypes.c_uint32), ("defer_after", ctypes.c_uint32),
                ("ts_start", ctypes.c_uint64), ("hbm_cap_bytes", ctypes.c_uint64), ("wait_limit_us", ctypes.c_uint64)]


_P = ctypes.c_void_p
_S = ctypes.c_int32
_SIGS = {
    "cc_version": (ctypes.c_char_p, []),
    "cc_strerror": (ctypes.c_char_p, [_S]),
    "cc_last_error": (ctypes.c_char_p, [_P]),
    "cc_init": (_S, [ctypes.POINTER(_P), ctypes.POINTER(cc_config)]),
    "cc_destroy": (_S, [_P]),
    "cc_create_table": (_S, [_P, ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]),
    "cc_load": (_S, [_P, ctypes.c_uint32, _P, ctypes.c_uint64, ctypes.c_int]),
    "cc_read_table": (_S, [_P, ctypes.c_uint32, _P, ctypes.c_int]),
    "cc_check_batch": (_S, [ctypes.c_uint32, _P, _P, _P, ctypes.c_uint64, _P, ctypes.c_uint64, ctypes.c_int]),
    "cc_submit_batch": (_S, [_P, _P, ctypes.c_uint64, _P, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                             ctypes.POINTER(ctypes.c_uint64)]),
    "cc_submit_batch_keyed": (_S, [_P, _P, ctypes.c_uint64, _P, ctypes.c_uint64, _P, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_uint64)]),
    "cc_create_index": (_S, [_P, ctypes.c_uint32, _P, ctypes.c_uint64]),
    "cc_fetch_rows": (_S, [_P, ctypes.c_uint64, _P]),
    "cc_engine_plan": (_S, [_P, ctypes.c_uint64, _P, _P, _P, _P]),
    "cc_run": (_S, [_P, ctypes.c_uint64, ctypes.POINTER(cc_run_params)]),
    "cc_check_run_params": (_S, [ctypes.c_int, ctypes.POINTER(cc_run_params)]),
    "cc_fetch_outcomes": (_S, [_P, ctypes.c_uint64, _P, _P, ctypes.c_int]),
    "cc_stats": (_S, [_P, ctypes.c_uint64, _P, ctypes.c_uint32]),
    "cc_set_arrivals": (_S, [_P, ctypes.c_uint64, _P, ctypes.c_uint64]),
    "cc_release_batch": (_S, [_P, ctypes.c_uint64]),
    "cc_run_static": (_S, [_P, _P, ctypes.c_uint64, _P, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(cc_run_params),
                           _P, _P, _P, ctypes.c_uint32]),
    "cc_device_info": (_S, [_P, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]),
    "cc_probe_indices": (_S, [_P, ctypes.c_int, ctypes.c_uint64, _P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]),
    "cc_probe": (_S, [_P, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                      ctypes.POINTER(ctypes.c_double)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class CCError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{lib.cc_strerror(status).decode()} ({status}): {message}")
        self.status = status
        self.message = message


def _check(st: int, ctx=None):
    if st != CC_OK:
        raise CCError(st, (lib.cc_last_error(ctx) or b"").decode())


def _host(a: np.ndarray, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a) -> int:
    if hasattr(a, "data_ptr"):
        return int(a.data_ptr())
    return int(a.ctypes.data)


# ---- entry points -----------------------------------------------------------

def cc_version() -> str:
    return lib.cc_version().decode()


def cc_strerror(status: int) -> str:
    return lib.cc_strerror(status).decode()


def cc_last_error(ctx=None) -> str:
    return (lib.cc_last_error(ctx) or b"").decode()


def cc_init(device: int = 0, stream=None):
    """Create a context; ``stream`` is a hipStream_t handle (int) or None."""
    ctx = _P()
    cfg = cc_config(device, 0, stream)
    _check(lib.cc_init(ctypes.byref(ctx), ctypes.byref(cfg)))
    return ctx


def cc_destroy(ctx) -> None:
    _check(lib.cc_destroy(ctx))


def cc_device_info(ctx):
    n_cu, khz = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib.cc_device_info(ctx, ctypes.byref(n_cu), ctypes.byref(khz)), ctx)
    return int(n_cu.value), int(khz.value)


PROBES = {"stream": 0, "gather": 1, "gather_plain": 2, "scatter": 3, "atomic": 4, "same_word": 5,
          "wave_counter": 6, "handoff": 7, "commit_handoff": 8, "engine_handoff": 9}


def cc_probe(ctx, kind, footprint_bytes: int, n_ops: int, peer: int = 1) -> float:
    """Run one memory micro-benchmark; returns its kernel time in ms."""
    if isinstance(kind, str):
        kind = PROBES[kind]
    ms = ctypes.c_double()
    _check(lib.cc_probe(ctx, kind, footprint_bytes, n_ops, peer, ctypes.byref(ms)), ctx)
    return float(ms.value)


def cc_probe_indices(ctx, kind, footprint_bytes: int, indices: np.ndarray) -> float:
    """Run the gather / scatter / atomic probe at the given word indices; returns its kernel time in ms."""
    if isinstance(kind, str):
        kind = PROBES[kind]
    idx = _host(indices, np.uint64)
    ms = ctypes.c_double()
    _check(lib.cc_probe_indices(ctx, kind, footprint_bytes, _ptr(idx), len(idx), ctypes.byref(ms)), ctx)
    return float(ms.value)


def cc_create_table(ctx, n_rows: int, n_fields: int) -> int:
    tid = ctypes.c_uint32()
    _check(lib.cc_create_table(ctx, n_rows, n_fields, ctypes.byref(tid)), ctx)
    return int(tid.value)


def cc_load(ctx, table_id: int, rows) -> None:
    """Copy a (n_rows, n_fields) int64 array (numpy, or a device tensor) into a table."""
    on_dev = hasattr(rows, "data_ptr")
    if not on_dev:
        rows = _host(rows, np.int64)
    _check(lib.cc_load(ctx, table_id, _ptr(rows), int(rows.shape[0]), int(on_dev)), ctx)


def cc_read_table(ctx, table_id: int, out) -> None:
    """Copy a table into ``out`` (a C-contiguous int64 numpy array or device tensor of the table's shape)."""
    on_dev = hasattr(out, "data_ptr")
    if not on_dev:
        assert out.dtype == np.int64 and out.flags["C_CONTIGUOUS"]
    _check(lib.cc_read_table(ctx, table_id, _ptr(out), int(on_dev)), ctx)


def cc_check_batch(table_shapes, txns: np.ndarray, ops: np.ndarray, scheme: int) -> int:
    """Host-only validation; returns the cc_status cc_submit_batch would give."""
    rows = np.array([s[0] for s in table_shapes], np.uint64)
    fields = np.array([s[1] for s in table_shapes], np.uint32)
    txns = _host(txns, TXN_DTYPE)
    ops = _host(ops, OP_DTYPE)
    return int(lib.cc_check_batch(len(rows), _ptr(rows), _ptr(fields), _ptr(txns), len(txns), _ptr(ops), len(ops),
                                  scheme))


def _count(a, itemsize: int) -> int:
    """Records in a host array (its length) or a device tensor (its bytes / the record size)."""
    if hasattr(a, "data_ptr"):
        nbytes = a.numel() * a.element_size()
        assert nbytes % itemsize == 0, "device array is not a whole number of records"
        return nbytes // itemsize
    return len(a)


def cc_submit_batch(ctx, txns, ops, scheme: int) -> int:
    """Submit host arrays (numpy, TXN_DTYPE / OP_DTYPE) or device tensors holding the same records."""
    on_dev = hasattr(txns, "data_ptr")
    assert on_dev == hasattr(ops, "data_ptr"), "txns and ops must both be host arrays or both device tensors"
    if not on_dev:
        txns = _host(txns, TXN_DTYPE)
        ops = _host(ops, OP_DTYPE)
    bid = ctypes.c_uint64()
    _check(lib.cc_submit_batch(ctx, _ptr(txns), _count(txns, 16), _ptr(ops), _count(ops, 16), scheme, int(on_dev),
                               ctypes.byref(bid)), ctx)
    return int(bid.value)


def cc_submit_batch_keyed(ctx, txns, ops, op_keys, scheme: int) -> int:
    on_dev = hasattr(txns, "data_ptr")
    assert on_dev == hasattr(ops, "data_ptr") == hasattr(op_keys, "data_ptr")
    if not on_dev:
        txns = _host(txns, TXN_DTYPE)
        ops = _host(ops, OP_DTYPE)
        op_keys = _host(op_keys, np.int64)
    assert _count(op_keys, 8) == _count(ops, 16)
    bid = ctypes.c_uint64()
    _check(lib.cc_submit_batch_keyed(ctx, _ptr(txns), _count(txns, 16), _ptr(ops), _count(ops, 16), _ptr(op_keys),
                                     scheme, int(on_dev), ctypes.byref(bid)), ctx)
    return int(bid.value)


def cc_check_run_params(scheme: int, params: cc_run_params | None = None) -> int:
    """Host-only check of run parameters; returns the cc_status cc_run would give before any device work."""
    p = params if params is not None else run_params()
    return int(lib.cc_check_run_params(scheme, ctypes.byref(p)))


def cc_create_index(ctx, table_id: int, keys: np.ndarray) -> None:
    keys = _host(keys, np.int64)
    _check(lib.cc_create_index(ctx, table_id, _ptr(keys), len(keys)), ctx)


def cc_fetch_rows(ctx, batch_id: int, n_ops: int) -> np.ndarray:
    rows = np.zeros(max(n_ops, 1), np.uint32)
    _check(lib.cc_fetch_rows(ctx, batch_id, _ptr(rows)), ctx)
    return rows[:n_ops]


def cc_engine_plan(ctx, batch_id: int):
    """(engine rows as global row ids, engine transactions, used by default) of a submitted batch."""
    rows = np.zeros(32, np.uint32)
    n_rows, n_txns, dflt = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_int()
    _check(lib.cc_engine_plan(ctx, batch_id, _ptr(rows), ctypes.byref(n_rows), ctypes.byref(n_txns),
                              ctypes.byref(dflt)), ctx)
    return rows[:n_rows.value].copy(), int(n_txns.value), bool(dflt.value)


def run_params(lanes_per_txn=0, waves_per_wg=0, grid=0, mode=CC_MODE_PLAIN, max_attempts=0, max_epochs=0,
               flags=0, backoff_ns=0, defer_after=0, ts_start=0, hbm_cap_bytes=0, wait_limit_us=0) -> cc_run_params:
    return cc_run_params(lanes_per_txn, waves_per_wg, grid, mode, max_attempts, max_epochs, flags, backoff_ns,
                         defer_after, ts_start, hbm_cap_bytes, wait_limit_us)


def cc_run(ctx, batch_id: int, params: cc_run_params | None = None) -> None:
    p = params if params is not None else run_params()
    _check(lib.cc_run(ctx, batch_id, ctypes.byref(p)), ctx)


def cc_fetch_outcomes(ctx, batch_id: int, per_txn=None, per_op_read=None) -> None:
    """Copy outcomes into ``per_txn`` (OUTCOME_DTYPE array) and read values into ``per_op_read`` (int64)."""
    on_dev = int(hasattr(per_txn, "data_ptr") or hasattr(per_op_read, "data_ptr"))
    p1 = _ptr(per_txn) if per_txn is not None else None
    p2 = _ptr(per_op_read) if per_op_read is not None else None
    _check(lib.cc_fetch_outcomes(ctx, batch_id, p1, p2, on_dev), ctx)


def cc_set_arrivals(ctx, batch_id: int, arrival_ns: np.ndarray) -> None:
    a = _host(arrival_ns, np.int64)
    _check(lib.cc_set_arrivals(ctx, batch_id, _ptr(a), len(a)), ctx)


def cc_stats(ctx, batch_id: int) -> dict:
    c = np.zeros(CC_N_STATS, np.uint64)
    _check(lib.cc_stats(ctx, batch_id, _ptr(c), CC_N_STATS), ctx)
    return {n: int(c[i]) for i, n in enumerate(STAT_NAMES)}


def cc_run_static(ctx, txns, ops, scheme: int, params: cc_run_params | None = None, per_txn=None,
                  per_op_read=None) -> dict:
    """Allocation-free run of a device-resident batch (device tensors of ABI structs as bytes) into the
    caller's device output tensors; returns the run's statistics."""
    n_txns, n_ops = _count(txns, TXN_DTYPE.itemsize), _count(ops, OP_DTYPE.itemsize)
    ctr = np.zeros(CC_N_STATS, np.uint64)
    p = ctypes.byref(params) if params is not None else None
    _check(lib.cc_run_static(ctx, _ptr(txns), n_txns, _ptr(ops), n_ops, scheme, p, _ptr(per_txn),
                             _ptr(per_op_read), _ptr(ctr), CC_N_STATS), ctx)
    return {k: int(v) for k, v in zip(STAT_NAMES, ctr)}


def cc_release_batch(ctx, batch_id: int) -> None:
    _check(lib.cc_release_batch(ctx, batch_id), ctx)


# ---- packing of workload batches into the ABI's arrays ---------------------

def pack_batch(batch):
    """(txns, ops) structured arrays of a workload.Batch, in the ABI's layout."""
    txns = np.zeros(batch.n_txns, TXN_DTYPE)
    txns["first_op"] = batch.first_op
    txns["n_ops"] = batch.n_ops
    ops = np.zeros(batch.total_ops, OP_DTYPE)
    ops["row"] = batch.row
    ops["table"] = batch.table
    ops["field"] = batch.field
    ops["kind"] = batch.kind
    ops["arg"] = batch.arg
    return txns, ops


class Engine:
    """A context with its tables loaded; thin convenience over the cc_* calls."""

    def __init__(self, tables, device: int = 0, stream=None):
        self.ctx = cc_init(device, stream)
        self.indexed = set()
        self.shapes = [tuple(t.shape) for t in tables]
        self.ids = [cc_create_table(self.ctx, int(s[0]), int(s[1])) for s in self.shapes]
        for i, t in zip(self.ids, tables):
            cc_load(self.ctx, i, t)

    def load(self, tables):
        for i, t in zip(self.ids, tables):
            cc_load(self.ctx, i, t)

    def tables(self):
        out = []
        for i, s in zip(self.ids, self.shapes):
            a = np.empty(s, np.int64)
            cc_read_table(self.ctx, i, a)
            out.append(a)
        return out

    def submit(self, batch, scheme) -> int:
        if isinstance(scheme, str):
            scheme = SCHEMES[scheme]
        txns, ops = pack_batch(batch)
        return cc_submit_batch(self.ctx, txns, ops, scheme)

    def submit_device(self, batch, scheme, device="cuda", keys=None) -> int:
        """Submit through device memory: the ABI arrays are copied into torch tensors on the GPU first
        and the library validates and packs them there (on_device = 1)."""
        import torch
        if isinstance(scheme, str):
            scheme = SCHEMES[scheme]
        txns, ops = pack_batch(batch)
        if keys is not None:
            ops["row"][np.isin(ops["table"], sorted(self.indexed))] = 0
        as_dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.uint8)).to(device)
        dt, do = as_dev(txns), as_dev(ops)
        if keys is None:
            return cc_submit_batch(self.ctx, dt, do, scheme)
        return cc_submit_batch_keyed(self.ctx, dt, do, as_dev(np.asarray(keys, np.int64)), scheme)

    def create_index(self, table_id, keys):
        cc_create_index(self.ctx, self.ids[table_id], keys)
        self.indexed.add(int(table_id))

    def submit_keyed(self, batch, op_keys, scheme) -> int:
        """Submit with rows named by key on tables that have an index (their ops' row fields are sent as 0)."""
        if isinstance(scheme, str):
            scheme = SCHEMES[scheme]
        txns, ops = pack_batch(batch)
        ops["row"][np.isin(ops["table"], sorted(self.indexed))] = 0
        return cc_submit_batch_keyed(self.ctx, txns, ops, op_keys, scheme)

    def rows(self, batch_id, n_ops):
        return cc_fetch_rows(self.ctx, batch_id, n_ops)

    def run(self, batch_id, **kw):
        cc_run(self.ctx, batch_id, run_params(**kw))
        return cc_stats(self.ctx, batch_id)

    def outcomes(self, batch_id, n_txns, n_ops):
        out = np.zeros(n_txns, OUTCOME_DTYPE)
        reads = np.zeros(n_ops, np.int64)
        cc_fetch_outcomes(self.ctx, batch_id, out if n_txns else None, reads if n_ops else None)
        return out, reads

    def release(self, batch_id):
        cc_release_batch(self.ctx, batch_id)

    def close(self):
        if self.ctx is not None:
            cc_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
