"""CPU oracle for the batch transaction engine -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the HIP engine: the serial
executor is plain C (``oracle.c``), the closed forms below are plain numpy.

Correctness criterion: every scheme guarantees serializable isolation (Section
3, "CC Schemes Migration and Implementation"; Section 4.1, "CC Scheme
Selection").  Non-deterministic schemes may legitimately produce different
outcomes for the same batch (Section 2, "conflict graph-based schemes being
deterministic, while others are non-deterministic"), so the oracle does not
predict one outcome.  It checks what is unique -- the set of committed
transactions, and the final tables of add-only batches (``final_add_only``,
a closed form that needs no order) -- and checks that the rest is valid: the
run's reported serial order, replayed serially, must reproduce every read value
and the final tables bit-exactly (``check_run``), and on tiny batches some
order out of all k! must do so (``bruteforce_count``).  The paper's own check
is acyclicity of a conflict graph built from an event log (Section 3.4,
"Measurements and Verification"); replaying a total order is a stronger form
of the same test.

The deterministic scheme (GaccO, conflict-graph ordering) does fix a unique
outcome: ``id_order_expected`` is the serial execution in transaction-id
order, compared element by element.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "perkey.c")]
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

# Outcome status values and op kinds, as the engine's interface defines them.
COMMITTED = 1
READ, ADD, COND_ADD, WRITE_SLOT = 0, 1, 2, 3

_P = ctypes.c_void_p


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP for the per-key checker) into oracle/liboracle.so."""
    if force or not os.path.exists(_SO) or any(os.path.getmtime(_SO) < os.path.getmtime(f) for f in _SRCS):
        tmp = _SO + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fopenmp", "-shared", "-fPIC", *_SRCS,
                        "-o", tmp], check=True)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        lib.oracle_replay.restype = ctypes.c_int
        lib.oracle_replay.argtypes = [ctypes.c_uint32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                      ctypes.c_uint64, _P, ctypes.c_uint64, _P]
        lib.oracle_bruteforce.restype = ctypes.c_int64
        lib.oracle_bruteforce.argtypes = [ctypes.c_uint32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                          ctypes.c_uint64, _P, ctypes.c_int, _P, ctypes.c_uint64]
        lib.oracle_perkey_check.restype = ctypes.c_int
        lib.oracle_perkey_check.argtypes = [ctypes.c_uint32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                            ctypes.c_uint64, ctypes.c_uint64, _P, _P, _P, _P, ctypes.c_int, _P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _batch_arrays(batch):
    return [np.ascontiguousarray(batch.first_op, np.uint64), np.ascontiguousarray(batch.n_ops, np.uint32),
            np.ascontiguousarray(batch.row, np.uint32), np.ascontiguousarray(batch.table, np.uint16),
            np.ascontiguousarray(batch.field, np.uint8), np.ascontiguousarray(batch.kind, np.uint8),
            np.ascontiguousarray(batch.arg, np.int64)]


def _table_args(tables):
    tabs = [np.ascontiguousarray(t, dtype=np.int64) for t in tables]
    n_rows = np.array([t.shape[0] for t in tabs], np.uint64)
    n_fields = np.array([t.shape[1] for t in tabs], np.uint32)
    ptrs = (ctypes.c_void_p * max(len(tabs), 1))(*[t.ctypes.data for t in tabs])
    return tabs, n_rows, n_fields, ptrs


_ERR = {-2: "row/field/table out of range", -3: "unknown op kind", -4: "WRITE_SLOT source not earlier",
        -5: "out of memory", -6: "bad argument", -7: "duplicate serial keys among committed transactions"}


def replay(tables, batch, order):
    """Serially execute ``batch`` transactions ``order`` (in that order) from ``tables``.

    Returns (final_tables, reads); reads[op] is the value op read, for ops of
    replayed transactions (other entries are 0).  Inputs are not modified.
    """
    lib = _load()
    tabs, n_rows, n_fields, ptrs = _table_args([np.array(t, dtype=np.int64, copy=True) for t in tables])
    arrs = _batch_arrays(batch)
    order = np.ascontiguousarray(order, dtype=np.int64)
    reads = np.zeros(max(batch.total_ops, 1), np.int64)
    rc = lib.oracle_replay(len(tabs), _ptr(n_rows), _ptr(n_fields), ptrs, *[_ptr(a) for a in arrs],
                           batch.n_txns, _ptr(order), len(order), _ptr(reads))
    if rc != 0:
        raise ValueError(f"oracle_replay: {_ERR.get(rc, rc)}")
    return tabs, reads[:batch.total_ops]


def serial_execute(tables, batch):
    """Execute every transaction of the batch serially in id order (no concurrency)."""
    return replay(tables, batch, np.arange(batch.n_txns, dtype=np.int64))


def id_order_expected(tables, batch):
    """Expected (final_tables, reads) of a conflict-graph-ordering run (GaccO).

    GaccO gathers every (transaction id, data item) access into an access
    table, orders each item's accesses by transaction id, and hands the item
    to its accessors one after the other in that order, reads and writes alike
    (Section 2, "Conflict Graph Ordering"; Section 3, "Conflict Graph
    Ordering").  Every conflict between two transactions is therefore ordered
    from the smaller id to the larger, the conflict graph is acyclic with the
    id order as a topological order, and the run is equivalent to executing
    the transactions serially in id order.  The outcome is unique (the scheme
    is deterministic), so parity is element by element against this replay.
    """
    return serial_execute(tables, batch)


def kset_ranks(batch):
    """GPUTx's rank of every transaction: its K-set (Section 2, "Conflict Graph Ordering").

    Conflicts are read-write, write-read and write-write accesses to the same
    item by two transactions, ordered by transaction id; they form a DAG, and a
    transaction's rank is its level in a topological sort of it: one more
    than the largest rank among the earlier transactions it conflicts with,
    0 if there are none.  Transactions of one rank never conflict, so a K-set
    runs without concurrency control, and executing the K-sets in rank order
    is equivalent to the id-order serial execution.  (Read literally, the
    per-item rule -- an item's k-th conflicting access gets rank k, the
    transaction takes its largest -- can put two conflicting transactions in
    one K-set; the DAG level is the rank that makes K-sets conflict-free.)
    An item is a (table, row); a transaction writes it if any of its
    operations on it writes.  Plain Python over the transactions in id order.
    """
    item_any = {}    # item -> largest rank of any earlier accessor
    item_write = {}  # item -> rank of the last earlier writer
    ranks = np.zeros(batch.n_txns, np.int64)
    for t in range(batch.n_txns):
        sl = batch.txn_slice(t)
        acc = {}
        for op in range(sl.start, sl.stop):
            item = (int(batch.table[op]), int(batch.row[op]))
            acc[item] = acc.get(item, False) or int(batch.kind[op]) != READ
        r = 0
        for item, writes in acc.items():
            before = item_any.get(item, -1) if writes else item_write.get(item, -1)
            r = max(r, before + 1)
        ranks[t] = r
        for item, writes in acc.items():
            item_any[item] = max(item_any.get(item, -1), r)
            if writes:
                item_write[item] = r
    return ranks


def resolve_keys(index_keys, batch, op_keys):
    """Rows that keyed operations name, through each table's index.

    The paper's index is a sorted array of a table's keys kept with the row
    ids and searched by binary search (Section 3.4, "Index"); the result of a
    lookup is simply the row that holds the key.  ``index_keys[t]`` is None
    for a table without an index, else an int64 array whose element i is row
    i's key (all distinct).  For an operation on an indexed table
    ``op_keys[op]`` is its key; other operations keep ``batch.row``.  Plain
    dictionary lookups, no search.  Raises KeyError for a key no row holds.
    """
    rows = np.array(batch.row, dtype=np.int64, copy=True)
    op_keys = np.asarray(op_keys, np.int64)
    for t, keys in enumerate(index_keys):
        if keys is None:
            continue
        where = {int(k): i for i, k in enumerate(np.asarray(keys, np.int64).tolist())}
        for op in np.nonzero(np.asarray(batch.table) == t)[0].tolist():
            rows[op] = where[int(op_keys[op])]
    return rows


def with_rows(batch, rows):
    """A copy of ``batch`` whose operations name ``rows``."""
    import copy
    b = copy.copy(batch)
    b.row = np.ascontiguousarray(rows, np.uint32)
    return b


def serial_order(status, serial_hi, serial_lo):
    """Committed transaction ids sorted by their (serial_hi, serial_lo) keys.

    Raises ValueError if two committed transactions report the same key (the
    reported order would not be a total order).
    """
    status = np.asarray(status)
    idx = np.nonzero(status == COMMITTED)[0]
    hi = np.asarray(serial_hi, np.uint64)[idx]
    lo = np.asarray(serial_lo, np.uint64)[idx]
    o = np.lexsort((lo, hi))
    hs, ls = hi[o], lo[o]
    if len(o) > 1 and np.any((hs[1:] == hs[:-1]) & (ls[1:] == ls[:-1])):
        raise ValueError("duplicate serial keys among committed transactions")
    return idx[o].astype(np.int64)


def final_add_only(tables, batch, committed=None):
    """Closed-form final tables for a batch of READ and ADD operations only.

    Adds commute, so the final value of every cell is its initial value plus
    the arguments of all committed ADDs on it, whatever the serial order.
    """
    if np.any((batch.kind != READ) & (batch.kind != ADD)):
        raise ValueError("closed form needs READ/ADD operations only")
    out = [np.array(t, dtype=np.int64, copy=True) for t in tables]
    txn_of_op = np.repeat(np.arange(batch.n_txns), batch.n_ops.astype(np.int64))
    m = batch.kind == ADD
    if committed is not None:
        m &= np.asarray(committed, bool)[txn_of_op]
    for t, tab in enumerate(out):
        mt = m & (batch.table == t)
        flat = tab.reshape(-1)
        idx = batch.row[mt].astype(np.int64) * tab.shape[1] + batch.field[mt].astype(np.int64)
        with np.errstate(over="ignore"):
            np.add.at(flat, idx, batch.arg[mt])
    return out


def bruteforce_count(tables, batch, txn_ids, got_reads, got_final) -> int:
    """Number of serial orders of ``txn_ids`` (k <= 8) reproducing the reads and final tables."""
    lib = _load()
    init, n_rows, n_fields, ptrs = _table_args(tables)
    fin, _, _, fptrs = _table_args(got_final)
    arrs = _batch_arrays(batch)
    txn_ids = np.ascontiguousarray(txn_ids, np.int64)
    got_reads = np.ascontiguousarray(got_reads, np.int64)
    rc = lib.oracle_bruteforce(len(init), _ptr(n_rows), _ptr(n_fields), ptrs, fptrs, *[_ptr(a) for a in arrs],
                               batch.n_txns, _ptr(txn_ids), len(txn_ids), _ptr(got_reads), batch.total_ops)
    if rc < 0:
        raise ValueError(f"oracle_bruteforce: {_ERR.get(int(rc), rc)}")
    return int(rc)


@dataclass
class CheckReport:
    ok: bool
    n_committed: int
    read_mismatches: int = 0
    table_mismatches: int = 0
    closed_form_ok: bool | None = None
    problems: list = field(default_factory=list)
    threads: int = 1

    def __str__(self):
        return (f"ok={self.ok} committed={self.n_committed} read_mismatch={self.read_mismatches} "
                f"table_mismatch={self.table_mismatches} closed_form={self.closed_form_ok} "
                f"problems={self.problems[:6]}")


def check_run(init_tables, batch, status, serial_hi, serial_lo, got_reads, got_final,
              require_all_committed=True) -> CheckReport:
    """Check one run of the engine against the definition of serializability.

    1. Every transaction committed (when required: the paper's batch model
       retries each transaction until it commits, Section 4.1).
    2. Committed transactions carry distinct serial keys.
    3. Replaying them serially in key order reproduces, element by element,
       every value the run reported as read, and the final tables.
    4. For add-only batches, the final tables equal the order-free closed form.
    """
    status = np.asarray(status)
    committed = status == COMMITTED
    rep = CheckReport(ok=True, n_committed=int(committed.sum()))
    if require_all_committed and not committed.all():
        rep.ok = False
        rep.problems.append(f"{int((~committed).sum())} transactions did not commit")
    try:
        order = serial_order(status, serial_hi, serial_lo)
    except ValueError as e:
        rep.ok = False
        rep.problems.append(str(e))
        return rep
    exp_final, exp_reads = replay(init_tables, batch, order)
    txn_of_op = np.repeat(np.arange(batch.n_txns), batch.n_ops.astype(np.int64))
    opm = committed[txn_of_op]
    got_reads = np.asarray(got_reads, np.int64)
    bad = np.nonzero(opm & (exp_reads != got_reads))[0]
    rep.read_mismatches = int(len(bad))
    for op in bad[:5]:
        rep.problems.append(f"txn {int(txn_of_op[op])} op {int(op)}: expected {int(exp_reads[op])} "
                            f"got {int(got_reads[op])}")
    for t, (e, g) in enumerate(zip(exp_final, got_final)):
        nb = int(np.count_nonzero(np.asarray(g, np.int64) != e))
        rep.table_mismatches += nb
        if nb:
            rep.problems.append(f"table {t}: {nb} cells differ from the serial replay")
    if np.all((batch.kind == READ) | (batch.kind == ADD)):
        cf = final_add_only(init_tables, batch, committed)
        rep.closed_form_ok = all(np.array_equal(c, np.asarray(g, np.int64)) for c, g in zip(cf, got_final))
        if not rep.closed_form_ok:
            rep.problems.append("final tables differ from the add-only closed form")
    rep.ok = rep.ok and rep.read_mismatches == 0 and rep.table_mismatches == 0 and rep.closed_form_ok is not False
    return rep


OE_WAREHOUSE_YTD = "warehouse ytd != sum of district ytd"
OE_CONSERVED = "customer balance + warehouse ytd not conserved"
OE_NEXT_O_ID = "district next_o_id growth != committed new-orders"
OE_ORDER_CNT = "stock order_cnt growth != committed order lines"
OE_SLOTS = "order slots: committed order ids of a district are not exactly its counter's range"
OE_SLOTS_UNTOUCHED = "order slots: a slot of an uncommitted new-order (or of no transaction) was written"


def order_entry_invariants(init_tables, final_tables, batch, committed) -> list:
    """Closed-form invariants of the order-entry workload; returns a list of violations.

    Each holds for every serial order of the committed transactions, so none
    needs the run's reported order (TPC-C's consistency conditions for the two
    transactions the paper runs, Section 4.1 "Benchmark Selection"):

    * warehouse ytd == sum of its districts' ytd (payments add the same amount to both);
    * sum(customer balance) + sum(warehouse ytd) is unchanged (payments move money);
    * district next-order-id growth == committed new-orders of that district;
    * total stock order-count growth == committed order lines;
    * the order slots of a district's k committed new-orders hold exactly the
      counter values init .. init+k-1, each once, because each new-order's
      order id is the pre-image of its district counter; slots of new-orders
      that did not commit keep their initial values.
    Every violation is reported with its own message (the OE_* constants).
    """
    from paper_2406_10158_amd import workload as wl  # table/field numbering only
    committed = np.asarray(committed, bool)
    out = []
    wh0, di0, cu0 = init_tables[wl.T_WAREHOUSE], init_tables[wl.T_DISTRICT], init_tables[wl.T_CUSTOMER]
    wh, di, cu, st = (np.asarray(final_tables[i], np.int64) for i in
                      (wl.T_WAREHOUSE, wl.T_DISTRICT, wl.T_CUSTOMER, wl.T_STOCK))
    st0 = init_tables[wl.T_STOCK]
    W = wh.shape[0]
    dsum = di[:, wl.D_YTD].reshape(W, wl.DISTRICTS_PER_W).sum(axis=1)
    if not np.array_equal(wh[:, wl.W_YTD], dsum):
        out.append(OE_WAREHOUSE_YTD)
    if cu[:, wl.C_BALANCE].sum() + wh[:, wl.W_YTD].sum() != cu0[:, wl.C_BALANCE].sum() + wh0[:, wl.W_YTD].sum():
        out.append(OE_CONSERVED)
    txn_of_op = np.repeat(np.arange(batch.n_txns), batch.n_ops.astype(np.int64))
    dop = (batch.table == wl.T_DISTRICT) & (batch.field == wl.D_NEXT_O_ID) & committed[txn_of_op]
    per_d = np.bincount(batch.row[dop].astype(np.int64), minlength=di.shape[0])
    if not np.array_equal(di[:, wl.D_NEXT_O_ID] - di0[:, wl.D_NEXT_O_ID], per_d):
        out.append(OE_NEXT_O_ID)
    lines = int(((batch.table == wl.T_ORDER_LINE) & (batch.field == wl.OL_AMOUNT) & committed[txn_of_op]).sum())
    if int(st[:, wl.S_ORDER_CNT].sum() - st0[:, wl.S_ORDER_CNT].sum()) != lines:
        out.append(OE_ORDER_CNT)
    # order slots: the transaction's district (its next-order-id op) and its slot row (its O_ID op)
    od0, od = init_tables[wl.T_ORDER], np.asarray(final_tables[wl.T_ORDER], np.int64)
    d_of = np.full(batch.n_txns, -1, np.int64)
    m = (batch.table == wl.T_DISTRICT) & (batch.field == wl.D_NEXT_O_ID)
    d_of[txn_of_op[m]] = batch.row[m]
    slot_of = np.full(batch.n_txns, -1, np.int64)
    m = (batch.table == wl.T_ORDER) & (batch.field == wl.O_ID)
    slot_of[txn_of_op[m]] = batch.row[m]
    owner = (slot_of >= 0) & (d_of >= 0)
    ok = True
    for d in np.unique(d_of[owner & committed]).tolist():
        got = np.sort(od[slot_of[owner & committed & (d_of == d)], wl.O_ID])
        want = np.arange(di0[d, wl.D_NEXT_O_ID], di0[d, wl.D_NEXT_O_ID] + len(got), dtype=np.int64)
        if not np.array_equal(got, want):
            ok = False
            break
    if not ok:
        out.append(OE_SLOTS)
    written = np.zeros(od.shape[0], bool)
    written[slot_of[owner & committed]] = True
    if not np.array_equal(od[~written], od0[~written]):
        out.append(OE_SLOTS_UNTOUCHED)
    return out


def check_run_perkey(init_tables, batch, status, serial_hi, serial_lo, got_reads, got_final,
                     require_all_committed=True, threads=0) -> CheckReport:
    """``check_run``'s question answered cell by cell on all host threads (C + OpenMP, ``perkey.c``).

    Every operation changes one cell as a function of that cell's previous
    value (a WRITE_SLOT also of the value its source operation reported, which
    is checked on the source's own cell), so the history of each cell can be
    replayed on its own, in serial-key order, and the cells in parallel.  A
    run passes here exactly when the serial replay of ``check_run`` accepts
    it.  ``threads`` <= 0: OpenMP's default (OMP_NUM_THREADS, else all cores).
    The report's ``problems`` name the lowest mismatching op and cell.
    """
    lib = _load()
    status = np.ascontiguousarray(status, np.uint32)
    committed = status == COMMITTED
    rep = CheckReport(ok=True, n_committed=int(committed.sum()))
    if require_all_committed and not committed.all():
        rep.ok = False
        rep.problems.append(f"{int((~committed).sum())} transactions did not commit")
    init, n_rows, n_fields, ptrs = _table_args(init_tables)
    fin, _, _, fptrs = _table_args(got_final)
    arrs = _batch_arrays(batch)
    hi = np.ascontiguousarray(serial_hi, np.uint64)
    lo = np.ascontiguousarray(serial_lo, np.uint64)
    reads = np.ascontiguousarray(got_reads, np.int64)
    res = np.zeros(6, np.int64)
    rc = lib.oracle_perkey_check(len(init), _ptr(n_rows), _ptr(n_fields), ptrs, fptrs, *[_ptr(a) for a in arrs],
                                 batch.n_txns, batch.total_ops, _ptr(status), _ptr(hi), _ptr(lo), _ptr(reads),
                                 int(threads), _ptr(res))
    if rc == -7:
        rep.ok = False
        rep.problems.append(_ERR[-7])
        return rep
    if rc != 0:
        raise ValueError(f"oracle_perkey_check: {_ERR.get(rc, rc)}")
    rep.read_mismatches, rep.table_mismatches = int(res[0]), int(res[1])
    rep.threads = int(res[5])
    if res[2] >= 0:
        rep.problems.append(f"op {int(res[2])}: read value differs from its cell's replay")
    if res[1]:
        rep.problems.append(f"{int(res[1])} cells differ from their replay (lowest touched: {int(res[3])})")
    rep.ok = rep.ok and rep.read_mismatches == 0 and rep.table_mismatches == 0
    return rep
