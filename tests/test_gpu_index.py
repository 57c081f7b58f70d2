"""Index lookups on the GPU: keyed batches under every scheme, both lookup methods.

Element by element: every row a lookup found (``cc_fetch_rows``) equals the
oracle's dictionary resolution of the key; the run itself is then checked
like any other (serial replay of the resolved batch in the reported order;
exact id-order replay for GaccO).  Index shapes cover single nodes, node and
level boundaries and extreme keys; misses must stop the run before anything
executes.
"""
import numpy as np
import pytest

import oracle
from helpers import SCHEMES, binding, check
from paper_2406_10158_amd import workload as wl

pytestmark = pytest.mark.gpu

ALL = SCHEMES + ["gacco", "gputx"]
METHODS = {"bsearch": 0, "tree": None}  # None: CC_RUN_INDEX_TREE


@pytest.fixture(scope="module", autouse=True)
def _announce(request):
    print(f"\n[gpu] module {request.module.__name__}", flush=True)


def _flags(method):
    b_ = binding()
    return b_.CC_RUN_INDEX_TREE if method == "tree" else 0


def run_keyed(tabs, b, keys_by_table, scheme, method, **params):
    """Run a keyed batch; returns (outcomes, reads, final tables, stats, rows found)."""
    b_ = binding()
    op_keys = wl.keyed_ops(b, keys_by_table)
    with b_.Engine(tabs) as eng:
        for t, k in enumerate(keys_by_table):
            if k is not None:
                eng.create_index(t, k)
        bid = eng.submit_keyed(b, op_keys, scheme)
        st = eng.run(bid, flags=params.pop("flags", 0) | _flags(method), **params)
        out, reads = eng.outcomes(bid, b.n_txns, b.total_ops)
        rows = eng.rows(bid, b.total_ops)
        final = eng.tables()
    return out, reads, final, st, rows


def check_keyed(tabs, b, keys_by_table, scheme, method, **params):
    out, reads, final, st, rows = run_keyed(tabs, b, keys_by_table, scheme, method, **params)
    exp_rows = oracle.resolve_keys(keys_by_table, b, wl.keyed_ops(b, keys_by_table))
    bad = np.nonzero(rows.astype(np.int64) != exp_rows)[0]
    assert len(bad) == 0, f"{len(bad)} lookups differ, first ops {bad[:5].tolist()}"
    rb = oracle.with_rows(b, exp_rows)
    if scheme in ("gacco", "gputx"):
        exp_fin, exp_reads = oracle.id_order_expected(tabs, rb)
        assert np.array_equal(reads, exp_reads)
        assert all(np.array_equal(g, e) for g, e in zip(final, exp_fin))
    else:
        rep = check(tabs, rb, out, reads, final)
        assert rep.ok, f"{scheme} {method}: {rep}"
    assert st["committed"] == b.n_txns
    return out, reads, final, st, rows


@pytest.mark.parametrize("method", ["bsearch", "tree"])
@pytest.mark.parametrize("scheme", ALL)
def test_keyed_kv(scheme, method):
    tabs, b = wl.kv_workload(n_rows=20_000, n_fields=4, n_txns=10_000, ops=16, theta=0.9, seed=31)
    keys = wl.index_keys(20_000, seed=31)
    *_, st = check_keyed(tabs, b, [keys], scheme, method)[:4]
    assert st["index_ns"] > 0


@pytest.mark.parametrize("method", ["bsearch", "tree"])
@pytest.mark.parametrize("n", [1, 15, 16, 17, 255, 256, 257, 4_097, 70_001])
def test_index_shapes_find_every_key(n, method):
    # one read of every row, by key; extreme keys included
    keys = wl.index_keys(n, seed=n)
    keys[0] = np.iinfo(np.int64).min
    if n > 1:
        keys[-1] = np.iinfo(np.int64).max - 1
    tabs = [wl.kv_table(n, 1)]
    ops = 4
    n_txns = (n + ops - 1) // ops
    row = np.arange(n_txns * ops) % n
    lengths = [min(ops, n - t * ops) for t in range(n_txns)]
    b = wl._pack(lengths, row[:sum(lengths)], np.zeros(n, np.int64), np.zeros(n, np.int64),
                 np.zeros(n, np.int64), np.zeros(n, np.int64), {})
    out, reads, final, st, rows = check_keyed(tabs, b, [keys], "occ", method)
    assert np.array_equal(rows, np.arange(n))
    assert np.array_equal(reads, 16 * np.arange(n))


@pytest.mark.parametrize("method", ["bsearch", "tree"])
def test_unknown_key_stops_the_run_before_anything_runs(method):
    b_ = binding()
    keys = np.array([10, 20, 30, 40, 50] * 1, np.int64)
    keys = np.concatenate([keys, np.arange(100, 100 + 35, dtype=np.int64)])  # 40 rows, two tree nodes + more
    tabs = [wl.kv_table(len(keys), 1)]
    b = wl.kv_batch(len(keys), 1, 30, ops=3, seed=5)
    for bad in (5, 25, 60, 99, 1 << 40, np.iinfo(np.int64).max):
        op_keys = wl.keyed_ops(b, [keys])
        op_keys[7] = bad
        with b_.Engine(tabs) as eng:
            eng.create_index(0, keys)
            bid = eng.submit_keyed(b, op_keys, "occ")
            with pytest.raises(b_.CCError) as e:
                eng.run(bid, flags=_flags(method))
            assert e.value.status == b_.CC_E_RANGE, bad
            assert np.array_equal(eng.tables()[0], tabs[0])


def test_keyed_submission_rules():
    b_ = binding()
    keys = wl.index_keys(100, seed=2)
    tabs = [wl.kv_table(100, 2)]
    with b_.Engine(tabs) as eng:
        eng.create_index(0, keys)
        # the same key twice, not adjacent, in one transaction
        b = wl._pack([3], np.array([1, 2, 1]), np.zeros(3, np.int64), np.array([0, 0, 1]), np.zeros(3, np.int64),
                     np.zeros(3, np.int64), {})
        with pytest.raises(b_.CCError) as e:
            eng.submit_keyed(b, wl.keyed_ops(b, [keys]), "occ")
        assert e.value.status == b_.CC_E_DUPROW
        # a row number on an indexed table's op
        txns, ops = b_.pack_batch(wl.kv_batch(100, 2, 2, ops=2, seed=3))
        ops["row"] = 5
        with pytest.raises(b_.CCError) as e:
            b_.cc_submit_batch_keyed(eng.ctx, txns, ops, np.zeros(len(ops), np.int64), b_.CC_OCC)
        assert e.value.status == b_.CC_E_INVAL
        # duplicate and reserved index keys
        with pytest.raises(b_.CCError):
            eng.create_index(0, np.zeros(100, np.int64))
        k2 = keys.copy()
        k2[3] = np.iinfo(np.int64).max
        with pytest.raises(b_.CCError):
            eng.create_index(0, k2)


@pytest.mark.parametrize("scheme", ["occ", "2pl_nw", "gacco", "gputx"])
def test_keyed_order_entry_with_an_index_on_customers(scheme):
    tabs, b = wl.order_entry_workload(8, 3_000, seed=7)
    keys = [None] * len(tabs)
    keys[wl.T_CUSTOMER] = wl.index_keys(tabs[wl.T_CUSTOMER].shape[0], seed=8)
    for method in ("bsearch", "tree"):
        out, reads, final, st, rows = check_keyed(tabs, b, keys, scheme, method)
        assert oracle.order_entry_invariants(tabs, final, b, out["status"] == 1) == []
        assert np.array_equal(rows.astype(np.int64), b.row.astype(np.int64))


def test_keyed_full_size_kv_config():
    # every lookup must return the row the generator drew the key from (keys are distinct)
    tabs, b = wl.kv_workload(seed=0)
    keys = wl.index_keys(tabs[0].shape[0], seed=0)
    for method in ("bsearch", "tree"):
        out, reads, final, st, rows = run_keyed(tabs, b, [keys], "occ", method)
        assert np.array_equal(rows.astype(np.int64), b.row.astype(np.int64))
        rep = check(tabs, b, out, reads, final)
        assert rep.ok, rep
        print(f"keyed full size {method}: index_ms={st['index_ns']/1e6:.3f} run_ms={st['run_ns']/1e6:.1f}")


@pytest.mark.parametrize("scheme", ["occ", "tictoc", "2pl_nw"])
def test_keyed_batches_in_epoch_and_serve_modes(scheme):
    # lookups run once per run before either mode's kernels; the resolved batch is then
    # checked like any other
    b_ = binding()
    tabs, b = wl.kv_workload(n_rows=30_000, n_fields=2, n_txns=8_000, ops=(2, 24), theta=0.8, seed=41)
    keys = wl.index_keys(30_000, seed=41)
    op_keys = wl.keyed_ops(b, [keys])
    exp_rows = oracle.resolve_keys([keys], b, op_keys)
    rb = oracle.with_rows(b, exp_rows)
    arrivals = np.sort(np.random.Generator(np.random.PCG64(42)).integers(0, 2_000_000, b.n_txns)).astype(np.int64)
    for mode in ("epoch", "serve"):
        with b_.Engine(tabs) as eng:
            eng.create_index(0, keys)
            bid = eng.submit_keyed(b, op_keys, scheme)
            if mode == "serve":
                b_.cc_set_arrivals(eng.ctx, bid, arrivals)
            st = eng.run(bid, mode=b_.CC_MODE_EPOCH if mode == "epoch" else b_.CC_MODE_SERVE,
                         flags=b_.CC_RUN_INDEX_TREE)
            out, reads = eng.outcomes(bid, b.n_txns, b.total_ops)
            rows = eng.rows(bid, b.total_ops)
            final = eng.tables()
        assert np.array_equal(rows.astype(np.int64), exp_rows), mode
        rep = check(tabs, rb, out, reads, final)
        assert rep.ok, (mode, rep)
        assert st["committed"] == b.n_txns and st["index_ns"] > 0
