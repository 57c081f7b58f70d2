"""Generator properties: determinism, distinct rows per transaction, Zipf frequencies, shapes."""
import numpy as np

from paper_2406_10158_amd import workload as wl


def test_same_seed_same_bytes():
    a = wl.kv_batch(10_000, 10, 2_000, ops=16, theta=0.9, seed=0)
    b = wl.kv_batch(10_000, 10, 2_000, ops=16, theta=0.9, seed=0)
    c = wl.kv_batch(10_000, 10, 2_000, ops=16, theta=0.9, seed=1)
    for k in ("row", "field", "kind", "arg", "first_op", "n_ops"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    assert not np.array_equal(a.row, c.row)


def test_rows_distinct_within_each_transaction():
    b = wl.kv_batch(1_000, 10, 5_000, ops=(2, 64), theta=0.99, seed=3)
    for t in range(0, b.n_txns, 7):
        r = b.row[b.txn_slice(t)]
        assert len(np.unique(r)) == len(r)
    assert b.n_ops.min() >= 2 and b.n_ops.max() <= 64
    assert int(b.first_op[-1]) + int(b.n_ops[-1]) == b.total_ops


def test_zipf_hottest_rank_frequency_matches_closed_form():
    n, theta, size = 1000, 0.9, 400_000
    rng = np.random.Generator(np.random.PCG64(0))
    keys = wl.draw_keys(rng, n, theta, size, scramble=False)
    p1 = 1.0 / sum(r ** -theta for r in range(1, n + 1))
    f1 = np.mean(keys == 0)
    assert abs(f1 - p1) < 5 * np.sqrt(p1 * (1 - p1) / size)
    p2 = 2 ** -theta * p1
    assert abs(np.mean(keys == 1) - p2) < 5 * np.sqrt(p2 / size)


def test_uniform_when_theta_zero_and_scramble_is_a_bijection():
    n = 10_007 * 3
    a = wl.scramble_multiplier(n)
    rows = (np.arange(n, dtype=np.uint64) * np.uint64(a)) % np.uint64(n)
    assert len(np.unique(rows)) == n
    rng = np.random.Generator(np.random.PCG64(1))
    k = wl.draw_keys(rng, 100, 0.0, 200_000)
    counts = np.bincount(k, minlength=100)
    assert counts.min() > 1700 and counts.max() < 2300


def test_read_ratio_and_arg_range():
    b = wl.kv_batch(100_000, 10, 20_000, ops=16, read_ratio=0.5, theta=0.6, seed=0)
    frac_read = np.mean(b.kind == wl.READ)
    assert abs(frac_read - 0.5) < 0.01
    adds = b.arg[b.kind == wl.ADD]
    assert adds.min() == -100 and adds.max() == 100
    assert np.all(b.arg[b.kind == wl.READ] == 0)
    assert b.field.max() == 9


def test_tiny_workload_shape():
    (tab,), b = wl.tiny_workload()
    assert tab.shape == (1024, 1) and np.array_equal(tab[:, 0], np.arange(1024))
    assert b.n_txns == 4096 and b.total_ops == 4096 * 4
    assert set(np.unique(b.arg[b.kind == wl.ADD])) == {1}


def test_order_entry_shape():
    tabs, b = wl.order_entry_workload(8, 400, seed=0)
    assert [t.shape[1] for t in tabs] == list(wl.OE_FIELDS)
    assert tabs[wl.T_STOCK].shape[0] == 8 * wl.STOCK_PER_W
    is_no = b.meta["is_new_order"]
    assert 0.4 < is_no.mean() < 0.6
    # ops on the same (table,row) are adjacent, and no (table,row,field) repeats within a txn
    for t in range(b.n_txns):
        s = b.txn_slice(t)
        keys = list(zip(b.table[s].tolist(), b.row[s].tolist()))
        seen = set()
        prev = None
        for k in keys:
            if k != prev:
                assert k not in seen
                seen.add(k)
            prev = k
        cells = list(zip(b.table[s].tolist(), b.row[s].tolist(), b.field[s].tolist()))
        assert len(set(cells)) == len(cells)
    # warehouse ytd equals the sum of district ytd initially
    assert np.array_equal(tabs[wl.T_WAREHOUSE][:, wl.W_YTD],
                          tabs[wl.T_DISTRICT][:, wl.D_YTD].reshape(8, 10).sum(1))


def test_hottest_row_chain_length_grows_with_theta():
    hs = []
    for th in (0.0, 0.6, 0.9, 0.99):
        b = wl.kv_batch(100_000, 10, 20_000, ops=16, theta=th, seed=0)
        hs.append(wl.hottest_row_writes(b)[1])
    assert hs == sorted(hs) and hs[-1] > 20 * hs[0]


def test_hottest_row_accesses_counts_transactions_not_ops():
    # two transactions touch row 3 (one of them with two fields), one touches row 5
    b = wl._pack([3, 2], np.array([3, 3, 7, 3, 5]), np.zeros(5, np.int64), np.array([0, 1, 0, 0, 0]),
                 np.array([1, 0, 0, 0, 1]), np.zeros(5, np.int64), {})
    assert wl.hottest_row_accesses(b) == (3, 2)
    assert wl.hottest_row_writes(b) == (3, 1)  # one of its accesses writes
    b2 = wl.kv_batch(100_000, 10, 20_000, ops=16, theta=0.9, seed=0)
    row, n = wl.hottest_row_accesses(b2)
    assert n >= wl.hottest_row_writes(b2)[1]
    assert n == len(set(np.repeat(np.arange(b2.n_txns), 16)[b2.row == row].tolist()))


def test_mixed_workload_follows_the_batch_rules():
    # row groups adjacent and never repeated, distinct fields per group, slot sources earlier in
    # the transaction, every kind present, lengths within the asked range, cells in range
    shapes = ((7, 2), (50, 4))
    tabs, b = wl.mixed_workload(shapes=shapes, n_txns=400, ops=(1, 12), theta=0.9, seed=4)
    assert [t.shape for t in tabs] == list(shapes)
    assert all(t.min() >= 0 and t.max() <= 60 for t in tabs)
    assert b.n_ops.min() >= 1 and b.n_ops.max() <= 12
    assert set(np.unique(b.kind).tolist()) == {wl.READ, wl.ADD, wl.COND_ADD, wl.WRITE_SLOT}
    for i in range(b.n_txns):
        sl = b.txn_slice(i)
        rows = list(zip(b.table[sl].tolist(), b.row[sl].tolist()))
        fields = b.field[sl].tolist()
        seen, prev = set(), None
        for j, (key, f) in enumerate(zip(rows, fields)):
            assert b.row[sl][j] < shapes[key[0]][0] and f < shapes[key[0]][1]
            if key != prev:
                assert key not in seen, (i, key)
                seen.add(key)
                group = set()
            assert f not in group
            group.add(f)
            prev = key
            if b.kind[sl][j] == wl.WRITE_SLOT:
                assert 0 <= (int(b.arg[sl][j]) & 0xFF) < j
