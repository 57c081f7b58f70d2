"""Seeded synthetic inputs for the batch transaction engine.

This module only draws inputs: tables, transactions and their operations.  It
holds none of the concurrency-control arithmetic and none of the operation
semantics; both the HIP engine and the CPU oracle consume what it returns.

Workload shapes follow the paper's evaluation setup (Section 4.1, "Benchmark
Selection"): YCSB-style key-value transactions of single-tuple accesses with
Zipfian keys, a write proportion, and TPC-C-style NewOrder / Payment
transactions.  Neither suite's own code is reproduced; these generators are
stand-ins with the same shapes, sizes and distributions.

Random numbers come from ``numpy.random.Generator(PCG64(seed))`` in a fixed
draw order, so a (config, seed) pair always yields the same bytes.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass, field as dc_field

import numpy as np

# Operation kinds (the numbering is part of the C-ABI, see include/cc.h).
READ, ADD, COND_ADD, WRITE_SLOT = 0, 1, 2, 3

# Order-entry table ids and field layouts.
T_WAREHOUSE, T_DISTRICT, T_CUSTOMER, T_ITEM, T_STOCK, T_ORDER, T_ORDER_LINE = range(7)
W_TAX, W_YTD = 0, 1
D_TAX, D_YTD, D_NEXT_O_ID = 0, 1, 2
C_DISCOUNT, C_BALANCE, C_YTD_PAYMENT, C_PAYMENT_CNT = 0, 1, 2, 3
I_PRICE = 0
S_QUANTITY, S_YTD, S_ORDER_CNT, S_REMOTE_CNT = 0, 1, 2, 3
O_ID, O_C_ID, O_OL_CNT = 0, 1, 2
OL_AMOUNT, OL_QUANTITY = 0, 1
OE_FIELDS = (2, 3, 4, 1, 4, 3, 2)
DISTRICTS_PER_W = 10
CUSTOMERS_PER_D = 3000
N_ITEMS = 100_000
STOCK_PER_W = 100_000
INIT_W_YTD = 30_000_000       # cents; equals 10 districts x INIT_D_YTD
INIT_D_YTD = 3_000_000
INIT_NEXT_O_ID = 3001
INIT_C_BALANCE = -1_000       # cents
INIT_S_QUANTITY_RANGE = (10, 100)


@dataclass
class Batch:
    """A batch of transactions in structure-of-arrays form.

    Transaction ``t`` owns operations ``first_op[t] .. first_op[t]+n_ops[t]-1``
    (in program order).  Operation ``i`` touches field ``field[i]`` of row
    ``row[i]`` of table ``table[i]`` with kind ``kind[i]`` and argument
    ``arg[i]``.
    """
    first_op: np.ndarray  # uint64 [n_txns]
    n_ops: np.ndarray     # uint32 [n_txns]
    row: np.ndarray       # uint32 [total_ops]
    table: np.ndarray     # uint16 [total_ops]
    field: np.ndarray     # uint8  [total_ops]
    kind: np.ndarray      # uint8  [total_ops]
    arg: np.ndarray       # int64  [total_ops]
    meta: dict = dc_field(default_factory=dict)

    @property
    def n_txns(self) -> int:
        return int(self.n_ops.shape[0])

    @property
    def total_ops(self) -> int:
        return int(self.row.shape[0])

    def txn_slice(self, t: int) -> slice:
        a = int(self.first_op[t])
        return slice(a, a + int(self.n_ops[t]))

    def subset(self, txn_ids) -> "Batch":
        """A new batch holding the given transactions, re-packed contiguously."""
        txn_ids = np.asarray(txn_ids, dtype=np.int64)
        n = self.n_ops[txn_ids].astype(np.uint32)
        first = np.zeros(len(txn_ids), dtype=np.uint64)
        if len(txn_ids):
            first[1:] = np.cumsum(n[:-1], dtype=np.uint64)
        lens = n.astype(np.int64)
        starts = self.first_op[txn_ids].astype(np.int64) if len(txn_ids) else np.zeros(0, np.int64)
        # op j of the k-th chosen transaction: starts[k] + j, laid out one transaction after another
        idx = np.repeat(starts - (np.cumsum(lens) - lens), lens) + np.arange(int(lens.sum()), dtype=np.int64)
        return Batch(first, n, self.row[idx].copy(), self.table[idx].copy(), self.field[idx].copy(),
                     self.kind[idx].copy(), self.arg[idx].copy(), dict(self.meta))


def _empty_batch() -> Batch:
    return Batch(np.zeros(0, np.uint64), np.zeros(0, np.uint32), np.zeros(0, np.uint32),
                 np.zeros(0, np.uint16), np.zeros(0, np.uint8), np.zeros(0, np.uint8),
                 np.zeros(0, np.int64))


# ----------------------------------------------------------------------------
# Key distributions
# ----------------------------------------------------------------------------

@functools.lru_cache(maxsize=8)
def zipf_cdf(n: int, theta: float) -> np.ndarray:
    """Cumulative probabilities of ranks 1..n with weight r^-theta (exact, normalised)."""
    if theta == 0.0:
        return np.arange(1, n + 1, dtype=np.float64) / n
    w = np.arange(1, n + 1, dtype=np.float64) ** (-float(theta))
    c = np.cumsum(w)
    c /= c[-1]
    c[-1] = 1.0
    return c


def zipf_p1(n: int, theta: float) -> float:
    """Probability of the hottest rank, 1 / zeta(n, theta)."""
    c = zipf_cdf(n, theta)
    return float(c[0])


def scramble_multiplier(n: int) -> int:
    """Multiplier A with gcd(A, n) == 1 so that rank -> (rank * A) mod n is a bijection."""
    if n <= 1:
        return 1
    a = 2654435761 % n
    if a == 0:
        a = 1
    while math.gcd(a, n) != 1:
        a += 1
    return a


def draw_keys(rng: np.random.Generator, n: int, theta: float, size: int, scramble: bool = True) -> np.ndarray:
    """Draw ``size`` row ids in [0, n) with Zipf(theta) popularity (theta=0 is uniform).

    Rank 0 is the hottest key.  With ``scramble`` the rank is mapped to a row by
    a fixed multiplicative bijection, so hot rows do not share cache lines.
    """
    if theta == 0.0:
        ranks = rng.integers(0, n, size=size, dtype=np.int64)
    else:
        u = rng.random(size)
        ranks = np.searchsorted(zipf_cdf(n, theta), u, side="right").astype(np.int64)
        np.minimum(ranks, n - 1, out=ranks)
    if not scramble:
        return ranks.astype(np.uint32)
    a = np.uint64(scramble_multiplier(n))
    return ((ranks.astype(np.uint64) * a) % np.uint64(n)).astype(np.uint32)


def rank_to_row(rank: int, n: int) -> int:
    return (rank * scramble_multiplier(n)) % n


def _distinct_rows(rng, n, theta, lengths, scramble=True, max_rounds=10_000):
    """Row ids per transaction, distinct within each transaction (redrawing duplicates)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    b = len(lengths)
    if b == 0:
        return np.zeros(0, np.uint32)
    m = int(lengths.max()) if b else 0
    if m > n:
        raise ValueError("a transaction needs more distinct rows than the table has")
    valid = np.arange(m)[None, :] < lengths[:, None]
    rows = np.zeros((b, m), dtype=np.int64)
    rows[valid] = draw_keys(rng, n, theta, int(valid.sum()), scramble)
    # Padding slots get values >= n, unique per column, so they never collide.
    pad = n + np.broadcast_to(np.arange(m), (b, m))
    rows[~valid] = pad[~valid]
    todo = np.arange(b)
    for _ in range(max_rounds):
        sub = rows[todo]
        order = np.argsort(sub, axis=1, kind="stable")
        ss = np.take_along_axis(sub, order, 1)
        dup_sorted = np.zeros_like(ss, dtype=bool)
        dup_sorted[:, 1:] = ss[:, 1:] == ss[:, :-1]
        if not dup_sorted.any():
            break
        has = dup_sorted.any(axis=1)
        todo = todo[has]
        order, dup_sorted, sub = order[has], dup_sorted[has], sub[has]
        dup = np.zeros_like(dup_sorted)
        np.put_along_axis(dup, order, dup_sorted, 1)
        sub[dup] = draw_keys(rng, n, theta, int(dup.sum()), scramble)
        rows[todo] = sub
    else:  # pragma: no cover - only reachable with absurd theta and tiny tables
        raise RuntimeError("could not draw distinct rows")
    return rows[valid].astype(np.uint32)


def _pack(lengths, row, table, field, kind, arg, meta) -> Batch:
    n_ops = np.asarray(lengths, dtype=np.uint32)
    first = np.zeros(len(n_ops), dtype=np.uint64)
    if len(n_ops) > 1:
        first[1:] = np.cumsum(n_ops[:-1], dtype=np.uint64)
    return Batch(first, n_ops, np.ascontiguousarray(row, np.uint32), np.ascontiguousarray(table, np.uint16),
                 np.ascontiguousarray(field, np.uint8), np.ascontiguousarray(kind, np.uint8),
                 np.ascontiguousarray(arg, np.int64), meta)


# ----------------------------------------------------------------------------
# Key-value (YCSB-style) workloads
# ----------------------------------------------------------------------------

def kv_table(n_rows: int, n_fields: int, identity: bool = False) -> np.ndarray:
    """Initial key-value table: value[r][f] = 16 r + f (or r when ``identity``)."""
    r = np.arange(n_rows, dtype=np.int64)[:, None]
    if identity:
        return np.repeat(r, n_fields, axis=1)
    return r * 16 + np.arange(n_fields, dtype=np.int64)[None, :]


def kv_batch(n_rows: int, n_fields: int, n_txns: int, ops=16, read_ratio: float = 0.5,
             theta: float = 0.0, arg_range=(-100, 100), seed: int = 0, scramble: bool = True,
             table_id: int = 0) -> Batch:
    """YCSB-style batch: each operation reads one field or adds a random int to it.

    ``ops`` is an int (fixed length) or a (lo, hi) pair (uniform length per txn).
    Rows are Zipf(theta) and distinct within a transaction; the field is
    uniform; an operation is a READ with probability ``read_ratio``, else an
    ADD whose argument is uniform on ``arg_range`` (inclusive).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if isinstance(ops, (tuple, list)):
        lengths = rng.integers(int(ops[0]), int(ops[1]) + 1, size=n_txns, dtype=np.int64)
    else:
        lengths = np.full(n_txns, int(ops), dtype=np.int64)
    total = int(lengths.sum())
    row = _distinct_rows(rng, n_rows, theta, lengths, scramble)
    field = rng.integers(0, n_fields, size=total, dtype=np.int64).astype(np.uint8)
    kind = np.where(rng.random(total) < read_ratio, READ, ADD).astype(np.uint8)
    arg = rng.integers(int(arg_range[0]), int(arg_range[1]) + 1, size=total, dtype=np.int64)
    arg[kind == READ] = 0
    table = np.full(total, table_id, dtype=np.uint16)
    meta = dict(workload="kv", n_rows=n_rows, n_fields=n_fields, theta=theta, read_ratio=read_ratio,
                seed=seed, ops=ops)
    return _pack(lengths, row, table, field, kind, arg, meta)


def tiny_workload(seed: int = 0):
    """1,024 rows x 1 field (value = row id); 4,096 txns x 4 ops, 50% read / 50% +1."""
    tab = kv_table(1024, 1, identity=True)
    b = kv_batch(1024, 1, 4096, ops=4, read_ratio=0.5, theta=0.0, arg_range=(1, 1), seed=seed)
    b.meta["workload"] = "tiny"
    return [tab], b


def kv_workload(n_rows=10_000_000, n_fields=10, n_txns=1_000_000, ops=16, read_ratio=0.5,
                theta=0.9, seed=0, scramble=True):
    tab = kv_table(n_rows, n_fields)
    b = kv_batch(n_rows, n_fields, n_txns, ops=ops, read_ratio=read_ratio, theta=theta,
                 arg_range=(-100, 100), seed=seed, scramble=scramble)
    return [tab], b


def hottest_row_writes(batch: Batch, table_id: int = 0) -> tuple[int, int]:
    """(row, number of write ops) of the most written row: the serial chain length H."""
    m = (batch.kind != READ) & (batch.table == table_id)
    if not m.any():
        return -1, 0
    rows, counts = np.unique(batch.row[m], return_counts=True)
    i = int(np.argmax(counts))
    return int(rows[i]), int(counts[i])


def index_keys(n_rows: int, seed: int = 0) -> np.ndarray:
    """Distinct random int64 keys, one per row (row i's key at index i), for a table with an index."""
    rng = np.random.Generator(np.random.PCG64(seed))
    keys = rng.integers(-(1 << 62), 1 << 62, size=n_rows, dtype=np.int64)
    while True:
        u, first = np.unique(keys, return_index=True)
        if len(u) == n_rows:
            return keys
        dup = np.ones(n_rows, bool)
        dup[first] = False
        keys[dup] = rng.integers(-(1 << 62), 1 << 62, size=int(dup.sum()), dtype=np.int64)


def keyed_ops(batch: Batch, keys_by_table) -> np.ndarray:
    """Per-op lookup keys: the key of the op's row for tables with keys (keys_by_table[t]), else 0."""
    out = np.zeros(batch.total_ops, np.int64)
    for t, keys in enumerate(keys_by_table):
        if keys is not None:
            m = batch.table == t
            out[m] = np.asarray(keys, np.int64)[batch.row[m].astype(np.int64)]
    return out


def hottest_row_accesses(batch: Batch, table_id: int = 0) -> tuple[int, int]:
    """(row, number of transactions accessing it) of the most accessed row, reads included."""
    m = batch.table == table_id
    if not m.any():
        return -1, 0
    txn_of_op = np.repeat(np.arange(batch.n_txns, dtype=np.int64), batch.n_ops.astype(np.int64))
    pairs = np.unique(batch.row[m].astype(np.int64) * batch.n_txns + txn_of_op[m])
    rows, counts = np.unique(pairs // batch.n_txns, return_counts=True)
    i = int(np.argmax(counts))
    return int(rows[i]), int(counts[i])


# ----------------------------------------------------------------------------
# Order-entry (TPC-C-style NewOrder / Payment) workloads
# ----------------------------------------------------------------------------

def mixed_workload(shapes=((40, 3), (300, 5)), n_txns=2_000, ops=(1, 16), theta=0.8,
                   kind_p=(0.35, 0.3, 0.2, 0.15), seed=0):
    """Small, contended tables and a batch that mixes every operation kind.

    ``shapes`` lists (rows, fields) per table; cells start uniform on [0, 60]
    so that conditional adds cross their threshold often.  A transaction's
    length is uniform on ``ops``; it is made of row groups: a (table, row) not
    used earlier in the transaction, Zipf(theta) within its table, with 1-3
    distinct fields whose operations are adjacent.  Kinds are drawn with
    probabilities ``kind_p`` = (READ, ADD, COND_ADD, WRITE_SLOT); a slot write
    takes its source uniformly among the transaction's earlier operations
    (the first operation of a transaction is never one).
    Returns (tables, batch).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    tables = [rng.integers(0, 61, size=(r, f), dtype=np.int64) for r, f in shapes]
    kp = np.asarray(kind_p, dtype=np.float64)
    kp = kp / kp.sum()
    lengths, row, table, field, kind, arg = [], [], [], [], [], []
    cap = sum(r * min(f, 3) for r, f in shapes)
    for _ in range(n_txns):
        want = int(rng.integers(int(ops[0]), int(ops[1]) + 1))
        if want > cap:
            raise ValueError("a transaction needs more cells than the tables offer")
        used = set()
        n = 0
        while n < want:
            t = int(rng.integers(0, len(shapes)))
            r = int(draw_keys(rng, shapes[t][0], theta, 1)[0])
            if (t, r) in used:
                continue
            used.add((t, r))
            g = int(rng.integers(1, min(shapes[t][1], want - n, 3) + 1))
            for f in rng.permutation(shapes[t][1])[:g]:
                k = int(rng.choice(4, p=kp))
                if k == WRITE_SLOT and n == 0:
                    k = ADD
                if k == READ:
                    a = 0
                elif k == ADD:
                    a = int(rng.integers(-50, 51))
                elif k == COND_ADD:
                    a = int(rng.integers(-30, 6))
                else:
                    a = slot_arg(int(rng.integers(0, n)), int(rng.integers(-1, 3)), int(rng.integers(-100, 101)))
                row.append(r); table.append(t); field.append(int(f)); kind.append(k); arg.append(a)
                n += 1
        lengths.append(n)
    b = _pack(lengths, np.array(row, np.uint32), np.array(table, np.uint16), np.array(field, np.uint8),
              np.array(kind, np.uint8), np.array(arg, np.int64), {})
    return tables, b


def slot_arg(src: int, mul: int, add: int) -> int:
    """Encode a WRITE_SLOT argument: value = read[src] * mul + add (see include/cc.h)."""
    if not (0 <= src < 256 and -(1 << 23) <= mul < (1 << 23) and -(1 << 31) <= add < (1 << 31)):
        raise ValueError("WRITE_SLOT argument out of range")
    v = (src & 0xFF) | ((mul & 0xFFFFFF) << 8) | ((add & 0xFFFFFFFF) << 32)
    if v >= 1 << 63:
        v -= 1 << 64
    return v


def order_entry_tables(n_warehouses: int, n_new_orders: int, n_order_lines: int, seed: int = 0):
    """Initial order-entry tables (int64 fixed-point cents), consistent with the invariants."""
    rng = np.random.Generator(np.random.PCG64(seed + 1_000_003))
    W = n_warehouses
    wh = np.zeros((W, OE_FIELDS[T_WAREHOUSE]), np.int64)
    wh[:, W_TAX] = rng.integers(0, 2001, size=W)            # basis points
    wh[:, W_YTD] = INIT_W_YTD
    di = np.zeros((W * DISTRICTS_PER_W, OE_FIELDS[T_DISTRICT]), np.int64)
    di[:, D_TAX] = rng.integers(0, 2001, size=len(di))
    di[:, D_YTD] = INIT_D_YTD
    di[:, D_NEXT_O_ID] = INIT_NEXT_O_ID
    nc = W * DISTRICTS_PER_W * CUSTOMERS_PER_D
    cu = np.zeros((nc, OE_FIELDS[T_CUSTOMER]), np.int64)
    cu[:, C_DISCOUNT] = rng.integers(0, 5001, size=nc)
    cu[:, C_BALANCE] = INIT_C_BALANCE
    cu[:, C_YTD_PAYMENT] = 1_000
    cu[:, C_PAYMENT_CNT] = 1
    it = np.zeros((N_ITEMS, OE_FIELDS[T_ITEM]), np.int64)
    it[:, I_PRICE] = rng.integers(100, 10_001, size=N_ITEMS)
    st = np.zeros((W * STOCK_PER_W, OE_FIELDS[T_STOCK]), np.int64)
    st[:, S_QUANTITY] = rng.integers(INIT_S_QUANTITY_RANGE[0], INIT_S_QUANTITY_RANGE[1] + 1, size=len(st))
    od = np.zeros((max(n_new_orders, 1), OE_FIELDS[T_ORDER]), np.int64)
    ol = np.zeros((max(n_order_lines, 1), OE_FIELDS[T_ORDER_LINE]), np.int64)
    return [wh, di, cu, it, st, od, ol]


def order_entry_workload(n_warehouses: int, n_txns: int, seed: int = 0, new_order_frac: float = 0.5,
                         remote_stock_p: float = 0.01, remote_customer_p: float = 0.15,
                         lines=(5, 15), quantity=(1, 8), amount=(1, 100_000)):
    """TPC-C-style NewOrder / Payment mix over seven tables.

    NewOrder (per transaction, in program order): read warehouse tax; read
    district tax and add 1 to its next order id (the pre-image is the order
    id); read the customer discount; per line read the item price and update
    the stock row (quantity by the replenishing conditional add, ytd, order
    count, remote count); then fill the transaction's own pre-assigned order
    slot and order-line slots from values read earlier (no inserts).
    Payment: add the amount to warehouse ytd and district ytd; subtract it
    from the customer's balance and add it to ytd-payment, payment count +1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    W = int(n_warehouses)
    is_no = rng.random(n_txns) < new_order_frac
    n_no = int(is_no.sum())
    n_lines = np.zeros(n_txns, np.int64)
    n_lines[is_no] = rng.integers(lines[0], lines[1] + 1, size=n_no)
    total_lines = int(n_lines.sum())
    lengths, row, table, field, kind, arg = [], [], [], [], [], []
    order_slot = 0
    line_slot = 0
    for t in range(n_txns):
        r, tb, fl, kd, ag = [], [], [], [], []

        def op(tab, rw, fld, k, a=0):
            r.append(rw); tb.append(tab); fl.append(fld); kd.append(k); ag.append(a)

        w = int(rng.integers(0, W))
        d = int(rng.integers(0, DISTRICTS_PER_W))
        drow = w * DISTRICTS_PER_W + d
        if is_no[t]:
            c = int(rng.integers(0, CUSTOMERS_PER_D))
            crow = drow * CUSTOMERS_PER_D + c
            nl = int(n_lines[t])
            items = rng.choice(N_ITEMS, size=nl, replace=False)
            remote = rng.random(nl) < remote_stock_p
            qty = rng.integers(quantity[0], quantity[1] + 1, size=nl)
            op(T_WAREHOUSE, w, W_TAX, READ)
            op(T_DISTRICT, drow, D_TAX, READ)
            src_oid = len(r)
            op(T_DISTRICT, drow, D_NEXT_O_ID, ADD, 1)
            op(T_CUSTOMER, crow, C_DISCOUNT, READ)
            price_src = []
            for l in range(nl):
                sw = w
                if remote[l] and W > 1:
                    sw = int(rng.integers(0, W - 1))
                    sw = sw + 1 if sw >= w else sw
                price_src.append(len(r))
                op(T_ITEM, int(items[l]), I_PRICE, READ)
                srow = sw * STOCK_PER_W + int(items[l])
                op(T_STOCK, srow, S_QUANTITY, COND_ADD, -int(qty[l]))
                op(T_STOCK, srow, S_YTD, ADD, int(qty[l]))
                op(T_STOCK, srow, S_ORDER_CNT, ADD, 1)
                if sw != w:
                    op(T_STOCK, srow, S_REMOTE_CNT, ADD, 1)
            op(T_ORDER, order_slot, O_ID, WRITE_SLOT, slot_arg(src_oid, 1, 0))
            op(T_ORDER, order_slot, O_C_ID, WRITE_SLOT, slot_arg(0, 0, crow))
            op(T_ORDER, order_slot, O_OL_CNT, WRITE_SLOT, slot_arg(0, 0, nl))
            order_slot += 1
            for l in range(nl):
                op(T_ORDER_LINE, line_slot, OL_AMOUNT, WRITE_SLOT, slot_arg(price_src[l], int(qty[l]), 0))
                op(T_ORDER_LINE, line_slot, OL_QUANTITY, WRITE_SLOT, slot_arg(0, 0, int(qty[l])))
                line_slot += 1
        else:
            h = int(rng.integers(amount[0], amount[1] + 1))
            if rng.random() < remote_customer_p:
                if W > 1:
                    cw = int(rng.integers(0, W - 1))
                    cw = cw + 1 if cw >= w else cw
                    cd = int(rng.integers(0, DISTRICTS_PER_W))
                else:
                    cw = w
                    cd = int(rng.integers(0, DISTRICTS_PER_W - 1))
                    cd = cd + 1 if cd >= d else cd
            else:
                cw, cd = w, d
            c = int(rng.integers(0, CUSTOMERS_PER_D))
            crow = (cw * DISTRICTS_PER_W + cd) * CUSTOMERS_PER_D + c
            op(T_WAREHOUSE, w, W_YTD, ADD, h)
            op(T_DISTRICT, drow, D_YTD, ADD, h)
            op(T_CUSTOMER, crow, C_BALANCE, ADD, -h)
            op(T_CUSTOMER, crow, C_YTD_PAYMENT, ADD, h)
            op(T_CUSTOMER, crow, C_PAYMENT_CNT, ADD, 1)
        lengths.append(len(r))
        row += r; table += tb; field += fl; kind += kd; arg += ag
    tables = order_entry_tables(W, order_slot, line_slot, seed)
    meta = dict(workload="order_entry", n_warehouses=W, seed=seed, n_new_orders=order_slot,
                n_order_lines=line_slot, is_new_order=is_no)
    b = _pack(lengths, np.array(row, np.int64), np.array(table, np.int64), np.array(field, np.int64),
              np.array(kind, np.int64), np.array(arg, np.int64), meta)
    return tables, b


# ----------------------------------------------------------------------------
# Serving streams: Poisson arrivals over a key-value / order-entry mix
# ----------------------------------------------------------------------------

def _gather_ops(sources, src, idx):
    """Operation index arrays of the transactions (sources[src[i]], idx[i]), concatenated in order.

    Returns (lengths, per-source op indices) so that the caller can gather
    each column from its source without a loop over transactions.
    """
    src = np.asarray(src, np.int64)
    idx = np.asarray(idx, np.int64)
    lengths = np.zeros(len(src), np.int64)
    firsts = np.zeros(len(src), np.int64)
    for j, bt in enumerate(sources):
        m = src == j
        lengths[m] = bt.n_ops[idx[m]].astype(np.int64)
        firsts[m] = bt.first_op[idx[m]].astype(np.int64)
    total = int(lengths.sum())
    starts = np.zeros(len(src), np.int64)
    if len(src) > 1:
        starts[1:] = np.cumsum(lengths[:-1])
    # op k of the result: source op firsts[t] + (k - starts[t]) of the transaction t that owns it
    owner = np.repeat(np.arange(len(src)), lengths)
    op_idx = firsts[owner] + (np.arange(total, dtype=np.int64) - starts[owner])
    return lengths, src[owner], op_idx


def concat_batches(parts):
    """One batch holding the given batches' transactions, in the given (batch, txn ids) order."""
    sources = []
    src, idx = [], []
    for bt, ids in parts:
        j = next((i for i, x in enumerate(sources) if x is bt), None)
        if j is None:
            sources.append(bt)
            j = len(sources) - 1
        ids = np.asarray(ids, np.int64).reshape(-1)
        src.append(np.full(len(ids), j, np.int64))
        idx.append(ids)
    src = np.concatenate(src) if src else np.zeros(0, np.int64)
    idx = np.concatenate(idx) if idx else np.zeros(0, np.int64)
    return _concat_sources(sources, src, idx)


def _concat_sources(sources, src, idx):
    lengths, op_src, op_idx = _gather_ops(sources, src, idx)
    cols = {}
    for name, dt in (("row", np.uint32), ("table", np.uint16), ("field", np.uint8), ("kind", np.uint8),
                     ("arg", np.int64)):
        out = np.zeros(len(op_idx), dt)
        for j, bt in enumerate(sources):
            m = op_src == j
            out[m] = getattr(bt, name)[op_idx[m]]
        cols[name] = out
    return _pack(lengths, cols["row"], cols["table"], cols["field"], cols["kind"], cols["arg"], {})


def _kv_chunk(args):
    n_rows, n_fields, n, ops, theta, seed = args
    return kv_batch(n_rows, n_fields, n, ops=ops, theta=theta, seed=seed)


def kv_parallel(n_rows: int, n_fields: int, n_txns: int, ops=16, theta: float = 0.0, seed: int = 0,
                workers: int = 8, chunk: int = 0):
    """Key-value transactions generated in chunks on `workers` processes (chunk i: seed * 7919 + i)."""
    import multiprocessing as mp
    chunk = chunk or max(20_000, -(-n_txns // (4 * max(workers, 1))))
    sizes = [min(chunk, n_txns - i) for i in range(0, n_txns, chunk)]
    jobs = [(n_rows, n_fields, n, ops, theta, seed * 7919 + i) for i, n in enumerate(sizes)]
    with mp.get_context("fork").Pool(max(1, min(workers, len(jobs)))) as pool:
        chunks = pool.map(_kv_chunk, jobs)
    src = np.concatenate([np.full(len(b.n_ops), j, np.int64) for j, b in enumerate(chunks)])
    idx = np.concatenate([np.arange(len(b.n_ops), dtype=np.int64) for b in chunks])
    return _concat_sources(chunks, src, idx)


def _oe_chunk(args):
    w, n, seed = args
    _, b = order_entry_workload(w, n, seed=seed)
    return b


def order_entry_parallel(n_warehouses: int, n_txns: int, seed: int = 0, workers: int = 8, chunk: int = 0):
    """Order-entry transactions generated in chunks on `workers` processes.

    Chunk i is ``order_entry_workload(W, ., seed + 1 + i)``; its order and
    order-line slots are moved past the previous chunks' slots, so that every
    new-order still owns its own slots.  The tables are the single-process
    generator's for ``seed`` with room for every slot.
    """
    import multiprocessing as mp
    chunk = chunk or max(20_000, -(-n_txns // (4 * max(workers, 1))))
    sizes = [min(chunk, n_txns - i) for i in range(0, n_txns, chunk)]
    jobs = [(n_warehouses, n, seed + 1 + i) for i, n in enumerate(sizes)]
    with mp.get_context("fork").Pool(max(1, min(workers, len(jobs)))) as pool:
        chunks = pool.map(_oe_chunk, jobs)
    no_off = lo_off = 0
    for b in chunks:
        m_o = b.table == T_ORDER
        m_l = b.table == T_ORDER_LINE
        b.row[m_o] += np.uint32(no_off)
        b.row[m_l] += np.uint32(lo_off)
        no_off += int(b.meta["n_new_orders"])
        lo_off += int(b.meta["n_order_lines"])
    tables = order_entry_tables(n_warehouses, no_off, lo_off, seed)
    src = np.concatenate([np.full(len(b.n_ops), j, np.int64) for j, b in enumerate(chunks)])
    idx = np.concatenate([np.arange(len(b.n_ops), dtype=np.int64) for b in chunks])
    out = _concat_sources(chunks, src, idx)
    out.meta = dict(workload="order_entry", n_warehouses=n_warehouses, seed=seed, n_new_orders=no_off,
                    n_order_lines=lo_off, is_new_order=np.concatenate([b.meta["is_new_order"] for b in chunks]))
    return tables, out


def serve_stream(n_arrivals: int, rate_per_s: float, kv_rows=10_000_000, kv_fields=10, kv_ops=(8, 32),
                 kv_theta=0.9, oe_warehouses=8, kv_frac=0.5, isolated_frac=0.0, seed=0, with_kv=True,
                 with_oe=True, arrivals_ns=None, kinds=None, workers=0, log=None):
    """A serving stream: tables, one batch in arrival order, arrival times (ns), and masks.

    Arrivals are a Poisson process of ``rate_per_s`` (exponential gaps).  Each
    arrival is a key-value transaction (table 0: ``kv_ops`` ops, Zipf
    ``kv_theta``) with probability ``kv_frac``, else an order-entry
    transaction (tables 1-7, ``oe_warehouses`` warehouses).  A fraction
    ``isolated_frac`` of the key-value transactions use private rows of a
    reserved range at the top of the key-value table that nothing else
    touches.  ``with_kv`` / ``with_oe`` drop one kind (keeping the others'
    arrival times), which gives the "alone" runs of a mixed stream.
    ``workers`` > 0 generates each part of a long stream (more than 200k
    arrivals of that kind) in chunks on that many processes; ``log`` (a
    callable) receives a line as each part is done.
    """
    rng = np.random.Generator(np.random.PCG64(seed + 7_000_001))
    if arrivals_ns is None:
        gaps = rng.exponential(1e9 / rate_per_s, size=n_arrivals)
        arrivals_ns = np.floor(np.cumsum(gaps)).astype(np.int64)
    if kinds is None:
        kinds = rng.random(n_arrivals) < kv_frac          # True: key-value
    n_kv = int(kinds.sum())
    n_oe = n_arrivals - n_kv
    n_iso = int(round(isolated_frac * n_kv))
    iso_rows_per = kv_ops[1] if isinstance(kv_ops, (tuple, list)) else int(kv_ops)
    reserved = n_iso * iso_rows_per
    shared_rows = kv_rows - reserved
    if workers and n_kv > 200_000 and n_iso == 0:
        kvb = kv_parallel(shared_rows, kv_fields, n_kv, ops=kv_ops, theta=kv_theta, seed=seed, workers=workers)
    else:
        kvb = kv_batch(shared_rows, kv_fields, n_kv, ops=kv_ops, theta=kv_theta, seed=seed)
    iso = np.zeros(n_kv, bool)
    if n_iso:
        iso_ids = rng.choice(n_kv, size=n_iso, replace=False)
        iso[iso_ids] = True
        for j, t in enumerate(np.sort(iso_ids)):
            sl = kvb.txn_slice(int(t))
            kvb.row[sl] = shared_rows + j * iso_rows_per + np.arange(sl.stop - sl.start, dtype=np.uint32)
    if log:
        log(f"key-value part: {n_kv} transactions")
    if workers and n_oe > 200_000:
        # long streams: order-entry chunks generated in parallel processes
        oe_tables, oeb = order_entry_parallel(oe_warehouses, n_oe, seed=seed + 1, workers=workers)
    else:
        oe_tables, oeb = order_entry_workload(oe_warehouses, max(n_oe, 1), seed=seed + 1)
    oeb.table = (oeb.table + 1).astype(np.uint16)
    if log:
        log(f"order-entry part: {n_oe} transactions")
    tables = [kv_table(kv_rows, kv_fields)] + oe_tables
    # interleave in arrival order: the a-th key-value arrival is kv transaction a', the
    # a-th order-entry arrival order-entry transaction a''
    kind_idx = np.where(kinds, np.cumsum(kinds) - 1, np.cumsum(~kinds) - 1).astype(np.int64)
    keep_m = (kinds & with_kv) | (~kinds & with_oe)
    keep = np.nonzero(keep_m)[0].astype(np.int64)
    src = np.where(kinds[keep], 0, 1).astype(np.int64)
    batch = _concat_sources([kvb, oeb], src, kind_idx[keep])
    is_kv = kinds[keep].astype(bool)
    is_iso = np.zeros(len(keep), bool)
    is_iso[is_kv] = iso[kind_idx[keep][is_kv]]
    batch.meta = dict(workload="serve", rate_per_s=rate_per_s, seed=seed, oe_warehouses=oe_warehouses,
                      is_new_order=np.zeros(len(keep), bool))
    return tables, batch, arrivals_ns[keep] if len(keep) else np.zeros(0, np.int64), dict(
        is_kv=is_kv, is_isolated=is_iso, arrivals_all=arrivals_ns, kinds=kinds)
