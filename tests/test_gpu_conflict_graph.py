"""The conflict-graph-ordering schemes on the GPU: GaccO and GPUTx.

Both are deterministic and equivalent to the transaction-id order, so every
run is compared element by element with the oracle's id-order replay
(``oracle.id_order_expected``): every read value, every cell of the final
tables, and the outcome records (all committed, one attempt each, serial key
(0, id) for GaccO and (K-set rank, id) for GPUTx, the ranks equal to
``oracle.kset_ranks``).  Cases cover the preprocessing (radix sort passes from 1 to 4,
ragged sort tiles, operations no transaction uses), the execution (lane
shapes including multi-word operation sets, grids, strict fences, one hot
row, row groups and slot writes of the order-entry workload) and the run
rules (plain mode only, ordered batches only).
"""
import numpy as np
import pytest

import oracle
from helpers import binding, run_batch
from paper_2406_10158_amd import workload as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _announce(request):
    print(f"\n[gpu] module {request.module.__name__}", flush=True)


# "gacco_shared": GaccO with CC_RUN_SHARED_READS (reads between two writes run together)
DETERMINISTIC = ["gacco", "gputx", "gacco_shared"]


def _sch(scheme):
    return "gacco" if scheme == "gacco_shared" else scheme


def _fl(scheme):
    return binding().CC_RUN_SHARED_READS if scheme == "gacco_shared" else 0


def run_exact(tabs, b, scheme="gacco", **params):
    params["flags"] = params.get("flags", 0) | _fl(scheme)
    out, reads, final, st = run_batch(tabs, b, _sch(scheme), **params)
    assert "error" not in st, st["error"]
    exp_fin, exp_reads = oracle.id_order_expected(tabs, b)
    n = b.n_txns
    assert np.all(out["status"] == oracle.COMMITTED)
    assert np.all(out["attempts"] == 1)
    if _sch(scheme) == "gacco":
        assert np.all(out["serial_hi"] == 0)
    else:
        ranks = oracle.kset_ranks(b)
        assert np.array_equal(out["serial_hi"].astype(np.int64), ranks)
        assert st["ksets"] == (int(ranks.max()) + 1 if n else 0)
        # the rank state shares the turn word below 2^20 transactions and 2^24 operations
        assert st["packed_state"] == int(n < (1 << 20) and b.total_ops < (1 << 24))
    assert np.array_equal(out["serial_lo"].astype(np.int64), np.arange(n))
    bad = np.nonzero(np.asarray(reads, np.int64) != exp_reads)[0]
    assert len(bad) == 0, f"{len(bad)} read values differ, first ops {bad[:5].tolist()}"
    for t, (g, e) in enumerate(zip(final, exp_fin)):
        nb = int(np.count_nonzero(np.asarray(g, np.int64) != e))
        assert nb == 0, f"table {t}: {nb} cells differ"
    assert st["committed"] == n and st["attempts"] == n
    return out, reads, final, st


@pytest.mark.parametrize("scheme", DETERMINISTIC)
def test_cg_tiny_config(scheme):
    tabs, b = wl.tiny_workload(seed=0)
    run_exact(tabs, b, scheme=scheme)


@pytest.mark.parametrize("theta", [0.0, 0.6, 0.9, 0.99])
@pytest.mark.parametrize("scheme", DETERMINISTIC)
def test_cg_kv(scheme, theta):
    tabs, b = wl.kv_workload(n_rows=200_000, n_fields=10, n_txns=30_001, ops=16, theta=theta, seed=1)
    out, reads, final, st = run_exact(tabs, b, scheme=scheme)
    print(f"{scheme} theta={theta}: prep_ms={st['prep_ns']/1e6:.3f} kernel_ms={st['kernel_ns']/1e6:.3f}")


@pytest.mark.parametrize("lanes,waves", [(1, 1), (1, 4), (4, 2), (4, 4), (16, 1), (16, 8), (64, 1), (64, 16)])
@pytest.mark.parametrize("scheme", DETERMINISTIC)
def test_cg_launch_shapes(scheme, lanes, waves):
    ops = (1, 16) if lanes == 1 else (2, 64)
    tabs, b = wl.kv_workload(n_rows=5_000, n_fields=4, n_txns=7_777, ops=ops, theta=0.9, seed=lanes * 31 + waves)
    run_exact(tabs, b, lanes_per_txn=lanes, waves_per_wg=waves, scheme=scheme)


@pytest.mark.parametrize("scheme", DETERMINISTIC)
def test_cg_grid_sizes(scheme):
    tabs, b = wl.kv_workload(n_rows=2_000, n_fields=2, n_txns=5_000, ops=8, theta=0.99, seed=2)
    for grid in (1, 3, 64, 4096):
        run_exact(tabs, b, grid=grid, waves_per_wg=2, scheme=scheme)


@pytest.mark.parametrize("scheme", DETERMINISTIC)
def test_cg_one_row_in_every_transaction(scheme):
    # every transaction touches row 0 (read or add) and three random rows: row
    # 0's chain is the whole batch, handed over 20k times in id order
    n = 20_000
    b = wl.kv_batch(1_000, 2, n, ops=4, read_ratio=0.5, arg_range=(-5, 5), seed=6)
    rows = b.row.reshape(n, 4)  # a view: rows stay distinct per transaction below
    rest = rows[:, 1:]
    t_zero, k_zero = np.nonzero(rest == 0)
    rest[t_zero, k_zero] = rows[t_zero, 0]
    rows[:, 0] = 0
    assert all(len(set(r)) == 4 for r in rows.tolist())
    tabs = [wl.kv_table(1_000, 2)]
    run_exact(tabs, b, lanes_per_txn=4, scheme=scheme)


@pytest.mark.parametrize("scheme", DETERMINISTIC)
def test_cg_edge_sizes(scheme):
    tabs = [wl.kv_table(64, 2)]
    b0 = wl.kv_batch(64, 2, 0, ops=4, seed=0)
    out, reads, final, st = run_batch(tabs, b0, _sch(scheme), flags=_fl(scheme))
    assert "error" not in st and st["committed"] == 0 and np.array_equal(final[0], tabs[0])
    run_exact(tabs, wl.kv_batch(64, 2, 1, ops=5, seed=1), scheme=scheme)
    b2 = wl.kv_batch(64, 2, 50, ops=(0, 3), seed=2)
    assert (b2.n_ops == 0).any()
    run_exact(tabs, b2, scheme=scheme)
    # transactions longer than 64 operations: operation sets span several words
    tabs3 = [wl.kv_table(4_000, 1)]
    b3 = wl.kv_batch(4_000, 1, 40, ops=(1, 256), theta=0.6, seed=3)
    assert b3.n_ops.max() > 192
    run_exact(tabs3, b3, lanes_per_txn=64, waves_per_wg=2, scheme=scheme)


@pytest.mark.parametrize("n_rows,n_ops", [(200, 3 * 4096 + 17), (60_000, 4096 - 3), (70_000, 5 * 4096 + 1)])
@pytest.mark.parametrize("scheme", DETERMINISTIC)
def test_cg_sort_tiles_and_passes(scheme, n_rows, n_ops):
    # 1 or 3 radix passes (row ids below 2^8 / 2^24), ragged last sort tile
    ops = 4
    b = wl.kv_batch(n_rows, 1, (n_ops + ops - 1) // ops, ops=ops, theta=0.9, seed=n_ops)
    run_exact([wl.kv_table(n_rows, 1)], b, scheme=scheme)


@pytest.mark.parametrize("scheme", DETERMINISTIC)
def test_cg_four_sort_passes(scheme):
    # total rows beyond 2^24 need a fourth 8-bit digit; the accessed rows sit
    # on both sides of 2^24
    n_rows = (1 << 24) + 1000
    rng = np.random.default_rng(9)
    n_txns, ops = 3_000, 4
    b = wl.kv_batch(1_000, 1, n_txns, ops=ops, seed=9)
    hot = np.array([5, (1 << 24) + 7, (1 << 24) + 999, 1 << 23], np.uint32)
    for t in range(n_txns):
        s = b.txn_slice(t)
        if t % 3:
            b.row[s] = rng.permutation(hot)
        else:
            r = rng.integers(0, n_rows, ops)
            while len(set(r.tolist())) < ops:
                r = rng.integers(0, n_rows, ops)
            b.row[s] = r
    run_exact([np.zeros((n_rows, 1), np.int64)], b, scheme=scheme)


@pytest.mark.parametrize("scheme", DETERMINISTIC)
def test_cg_unused_ops_stay_out_of_the_access_table(scheme):
    # ops no transaction refers to (gaps in the ops array) must not hold a turn
    b_ = binding()
    tabs = [wl.kv_table(100, 1)]
    b = wl.kv_batch(100, 1, 300, ops=3, theta=0.9, seed=11)
    txns, ops = b_.pack_batch(b)
    # spread the transactions out with a one-op gap after each; gap ops name row 0
    ops2 = np.zeros(len(ops) + b.n_txns, ops.dtype)
    txns2 = txns.copy()
    for t in range(b.n_txns):
        s = int(txns["first_op"][t])
        ops2[s + t: s + t + 3] = ops[s: s + 3]
        txns2["first_op"][t] = s + t
    eng = b_.Engine(tabs)
    try:
        bid = b_.cc_submit_batch(eng.ctx, txns2, ops2, b_.SCHEMES[_sch(scheme)])
        st = eng.run(bid, flags=_fl(scheme))
        out, reads = eng.outcomes(bid, b.n_txns, len(ops2))
        final = eng.tables()
    finally:
        eng.close()
    exp_fin, exp_reads = oracle.id_order_expected(tabs, b)
    used = np.concatenate([np.arange(int(txns2["first_op"][t]), int(txns2["first_op"][t]) + 3)
                           for t in range(b.n_txns)])
    assert np.array_equal(reads[used], exp_reads)
    assert np.array_equal(final[0], exp_fin[0])
    assert st["committed"] == b.n_txns


@pytest.mark.parametrize("warehouses", [1, 8])
@pytest.mark.parametrize("scheme", DETERMINISTIC)
def test_cg_order_entry(scheme, warehouses):
    tabs, b = wl.order_entry_workload(warehouses, 4_000, seed=warehouses)
    out, reads, final, st = run_exact(tabs, b, scheme=scheme)
    assert oracle.order_entry_invariants(tabs, final, b, np.ones(b.n_txns, bool)) == []


@pytest.mark.parametrize("scheme", DETERMINISTIC)
def test_cg_uneven_batch_shapes(scheme):
    # the batching workload's shape: 2..64 ops per transaction, Zipf 0.8
    tabs, b = wl.kv_workload(n_rows=100_000, n_fields=10, n_txns=16_384, ops=(2, 64), theta=0.8, seed=12)
    for lanes in (4, 16, 64):
        run_exact(tabs, b, lanes_per_txn=lanes, scheme=scheme)


@pytest.mark.parametrize("scheme", DETERMINISTIC)
def test_cg_strict_fences(scheme):
    b_ = binding()
    tabs, b = wl.kv_workload(n_rows=20_000, n_fields=4, n_txns=20_000, ops=16, theta=0.99, seed=7)
    run_exact(tabs, b, flags=b_.CC_RUN_STRICT_FENCES, scheme=scheme)


@pytest.mark.parametrize("scheme", DETERMINISTIC)
def test_cg_repeated_runs_accumulate(scheme):
    b_ = binding()
    tabs, b = wl.kv_workload(n_rows=5_000, n_fields=2, n_txns=3_000, ops=8, theta=0.9, seed=8)
    eng = b_.Engine(tabs)
    try:
        bid = eng.submit(b, _sch(scheme))
        eng.run(bid, flags=_fl(scheme))
        eng.run(bid, flags=_fl(scheme))
        out, reads = eng.outcomes(bid, b.n_txns, b.total_ops)
        final = eng.tables()
    finally:
        eng.close()
    mid, _ = oracle.id_order_expected(tabs, b)
    exp_fin, exp_reads = oracle.id_order_expected(mid, b)
    assert np.array_equal(reads, exp_reads)
    assert np.array_equal(final[0], exp_fin[0])


@pytest.mark.parametrize("scheme", DETERMINISTIC)
def test_cg_run_rules(scheme):
    b_ = binding()
    tabs, b = wl.kv_workload(n_rows=1_000, n_fields=2, n_txns=500, ops=4, theta=0.5, seed=10)
    eng = b_.Engine(tabs)
    try:
        bid = eng.submit(b, _sch(scheme))
        with pytest.raises(b_.CCError) as e:
            eng.run(bid, mode=b_.CC_MODE_EPOCH)
        assert e.value.status == b_.CC_E_INVAL
        with pytest.raises(b_.CCError) as e:
            eng.run(bid, flags=b_.CC_RUN_PRECHECK)
        assert e.value.status == b_.CC_E_INVAL
        with pytest.raises(b_.CCError) as e:
            eng.run(bid, flags=b_.CC_RUN_LATCH)  # a deterministic scheme has no latch variant
        assert e.value.status == b_.CC_E_INVAL
        if _sch(scheme) == "gputx":
            with pytest.raises(b_.CCError) as e:
                eng.run(bid, flags=b_.CC_RUN_SHARED_READS)  # shared reads are a GaccO option
            assert e.value.status == b_.CC_E_INVAL
        st = eng.run(bid, flags=_fl(scheme))  # the batch is still usable after the rejected runs
        assert st["committed"] == b.n_txns
    finally:
        eng.close()


@pytest.mark.parametrize("scheme", DETERMINISTIC)
def test_cg_full_size_kv_config(scheme):
    tabs, b = wl.kv_workload(seed=0)
    out, reads, final, st = run_exact(tabs, b, scheme=scheme)
    print(f"{scheme} full: run_ms={st['run_ns']/1e6:.1f} prep_ms={st['prep_ns']/1e6:.2f} "
          f"kernel_ms={st['kernel_ns']/1e6:.1f}")


def test_gputx_rank_state_in_its_own_word_for_large_batches():
    # 2^20 + 1000 transactions: too many for the packed rank state, so the rank pass keeps
    # the state in its own word next to a turn word of sorted positions
    tabs, b = wl.kv_workload(n_rows=200_000, n_fields=2, n_txns=(1 << 20) + 1000, ops=2, theta=0.8, seed=79)
    *_, st = run_exact(tabs, b, "gputx")
    assert st["packed_state"] == 0 and st["ksets"] > 10


@pytest.mark.parametrize("scheme", DETERMINISTIC)
def test_wait_limit_stops_the_run_and_the_context_recovers(scheme):
    # The bounded wait's stop path, forced from the host: with a 1 us limit a contended run
    # stops (every team leaves its wait and every kernel exits), the run reports
    # CC_E_LIVELOCK, and the next run of the same batch on reloaded tables matches the
    # id-order execution exactly.
    bb = binding()
    tabs, b = wl.kv_workload(n_rows=2_000, n_fields=2, n_txns=20_000, ops=8, theta=0.99, seed=77)
    print(f"[gpu] wait limit {scheme}", flush=True)
    with bb.Engine(tabs) as eng:
        bid = eng.submit(b, _sch(scheme))
        with pytest.raises(bb.CCError) as e:
            eng.run(bid, flags=_fl(scheme), wait_limit_us=1)
        assert e.value.status == bb.CC_E_LIVELOCK
        eng.load(tabs)
        st = eng.run(bid, flags=_fl(scheme))
        assert st["committed"] == b.n_txns
        out, reads = eng.outcomes(bid, b.n_txns, b.total_ops)
        final = eng.tables()
    exp_fin, exp_reads = oracle.id_order_expected(tabs, b)
    assert np.array_equal(np.asarray(reads, np.int64), exp_reads)
    assert all(np.array_equal(np.asarray(g, np.int64), x) for g, x in zip(final, exp_fin))


def test_wait_limit_is_rejected_for_the_other_schemes():
    bb = binding()
    tabs, b = wl.kv_workload(n_rows=1_000, n_fields=2, n_txns=100, ops=4, seed=78)
    with bb.Engine(tabs) as eng:
        bid = eng.submit(b, "occ")
        with pytest.raises(bb.CCError) as e:
            eng.run(bid, wait_limit_us=10)
        assert e.value.status == bb.CC_E_INVAL
        assert np.array_equal(eng.tables()[0], tabs[0])
