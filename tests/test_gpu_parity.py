"""GPU parity: every run of the HIP engine is checked against the CPU oracle.

Per run: all transactions commit, serial keys are distinct, the serial replay
in key order reproduces every read value and the final tables element by
element, and add-only batches end in the order-free closed form.  Special
cases pin outputs with no GPU input at all (single team = serial execution,
read-only batches, disjoint keys), and tiny batches are brute-forced.
"""
import functools

import numpy as np
import pytest

import oracle
from helpers import SCHEMES, binding, check, run_and_check, run_batch
from paper_2406_10158_amd import workload as wl

pytestmark = pytest.mark.gpu

IMPLEMENTED = SCHEMES
TICKETED = ["occ", "2pl_nw", "to", "mvcc", "2pl_wd"]  # serial key (0, counter)


@pytest.fixture(scope="module", autouse=True)
def _announce(request):
    print(f"\n[gpu] module {request.module.__name__}", flush=True)


@pytest.mark.parametrize("scheme", IMPLEMENTED)
def test_tiny_config(scheme):
    tabs, b = wl.tiny_workload(seed=0)
    out, reads, final, st = run_and_check(tabs, b, scheme)
    # the tiny config is add-only: final table is the closed form, independent of order
    assert np.array_equal(final[0], oracle.final_add_only(tabs, b)[0])


@pytest.mark.parametrize("scheme", IMPLEMENTED)
@pytest.mark.parametrize("theta", [0.0, 0.6, 0.9, 0.99])
def test_kv_parity(scheme, theta):
    tabs, b = wl.kv_workload(n_rows=200_000, n_fields=10, n_txns=30_001, ops=16, theta=theta, seed=1)
    out, reads, final, st = run_and_check(tabs, b, scheme)
    print(f"{scheme} theta={theta}: attempts={st['attempts']} kernel_ms={st['kernel_ns']/1e6:.3f}")


@pytest.mark.parametrize("scheme", IMPLEMENTED)
@pytest.mark.parametrize("lanes,waves", [(1, 1), (1, 4), (4, 2), (4, 4), (16, 1), (16, 8), (64, 1), (64, 16)])
def test_launch_shapes(scheme, lanes, waves):
    ops = (1, 16) if lanes == 1 else (2, 64)
    tabs, b = wl.kv_workload(n_rows=5_000, n_fields=4, n_txns=7_777, ops=ops, theta=0.9, seed=lanes * 31 + waves)
    run_and_check(tabs, b, scheme, lanes_per_txn=lanes, waves_per_wg=waves)


@pytest.mark.parametrize("scheme", IMPLEMENTED)
def test_grid_sizes(scheme):
    tabs, b = wl.kv_workload(n_rows=2_000, n_fields=2, n_txns=5_000, ops=8, theta=0.99, seed=2)
    for grid in (1, 3, 64, 4096):
        run_and_check(tabs, b, scheme, grid=grid, waves_per_wg=2)


@pytest.mark.parametrize("scheme", IMPLEMENTED)
def test_single_team_is_serial_execution(scheme):
    # one workgroup of one wavefront with one 64-lane team: transactions run one at a time in id
    # order, so the result is the oracle's own serial execution, with no GPU input to the oracle
    # (OCC without the hot-row engine, which runs the hottest rows' writers first)
    tabs, b = wl.kv_workload(n_rows=300, n_fields=3, n_txns=400, ops=(1, 40), theta=0.9, seed=3)
    f = binding().CC_RUN_NO_HOT_ENGINE if scheme == "occ" else 0
    out, reads, final, st = run_batch(tabs, b, scheme, lanes_per_txn=64, waves_per_wg=1, grid=1, flags=f)
    assert "error" not in st
    exp_final, exp_reads = oracle.serial_execute(tabs, b)
    assert np.array_equal(reads, exp_reads)
    assert np.array_equal(final[0], exp_final[0])
    assert st["attempts"] == b.n_txns  # zero aborts
    if scheme in TICKETED:
        assert np.all(np.diff(oracle.serial_order(out["status"], out["serial_hi"], out["serial_lo"])) == 1)
    assert check(tabs, b, out, reads, final).ok


@pytest.mark.parametrize("scheme", IMPLEMENTED)
def test_read_only_batch(scheme):
    tabs, b = wl.kv_workload(n_rows=50_000, n_fields=10, n_txns=20_000, ops=16, read_ratio=1.0, theta=0.99, seed=4)
    out, reads, final, st = run_and_check(tabs, b, scheme)
    assert np.array_equal(reads, 16 * b.row.astype(np.int64) + b.field.astype(np.int64))
    assert np.array_equal(final[0], tabs[0])


@pytest.mark.parametrize("scheme", IMPLEMENTED)
def test_disjoint_keys(scheme):
    n_txn, ops = 4_096, 8
    b = wl.kv_batch(n_txn * ops, 2, n_txn, ops=ops, seed=5)
    b.row[:] = np.random.default_rng(5).permutation(n_txn * ops).astype(np.uint32)
    tabs = [wl.kv_table(n_txn * ops, 2)]
    out, reads, final, st = run_and_check(tabs, b, scheme)
    assert np.array_equal(reads, 16 * b.row.astype(np.int64) + b.field.astype(np.int64))
    assert st["attempts"] == n_txn  # nothing conflicts, nothing aborts


@pytest.mark.parametrize("scheme", IMPLEMENTED)
def test_bruteforce_tiny_batches(scheme):
    # <= 7 transactions on 3 rows, all in one wavefront (1 lane each): every outcome must be one
    # of the k! serial executions
    for seed in range(12):
        tabs, b = wl.kv_workload(n_rows=3, n_fields=1, n_txns=7, ops=(1, 3), theta=0.0, seed=100 + seed)
        out, reads, final, st = run_batch(tabs, b, scheme, lanes_per_txn=1, waves_per_wg=1)
        assert "error" not in st
        assert np.all(out["status"] == 1)
        assert oracle.bruteforce_count(tabs, b, np.arange(b.n_txns), reads, final) >= 1
        assert check(tabs, b, out, reads, final).ok


@pytest.mark.parametrize("scheme", IMPLEMENTED)
def test_two_hot_rows_stress(scheme):
    # every transaction adds to both of two rows: a total order of 20k conflicting updates
    n = 20_000
    b = wl.kv_batch(2, 1, n, ops=2, read_ratio=0.3, arg_range=(-5, 5), seed=6)
    tabs = [wl.kv_table(2, 1)]
    out, reads, final, st = run_and_check(tabs, b, scheme, lanes_per_txn=4)
    # there was contention: aborts, or (OCC's hot-row engine) waits for a row
    assert st["attempts"] > n or st["engine_waits"] > 0


@pytest.mark.parametrize("scheme", IMPLEMENTED)
def test_edge_sizes(scheme):
    tabs = [wl.kv_table(64, 2)]
    # empty batch
    b0 = wl.kv_batch(64, 2, 0, ops=4, seed=0)
    out, reads, final, st = run_batch(tabs, b0, scheme)
    assert "error" not in st and st["committed"] == 0 and np.array_equal(final[0], tabs[0])
    # one transaction; a transaction with no ops among others
    b1 = wl.kv_batch(64, 2, 1, ops=5, seed=1)
    run_and_check(tabs, b1, scheme)
    b2 = wl.kv_batch(64, 2, 50, ops=(0, 3), seed=2)
    assert (b2.n_ops == 0).any()
    run_and_check(tabs, b2, scheme)
    # the largest transaction (256 ops) next to small ones
    tabs3 = [wl.kv_table(4_000, 1)]
    b3 = wl.kv_batch(4_000, 1, 40, ops=(1, 256), theta=0.6, seed=3)
    assert b3.n_ops.max() > 192
    run_and_check(tabs3, b3, scheme, lanes_per_txn=64, waves_per_wg=2)


@pytest.mark.parametrize("scheme", ["occ", "mvcc", "gacco", "gputx"])
def test_maximum_total_rows(scheme):
    # 2^28 rows in all (the limit): one table of 2^28 - 16 rows and one of 16. Row indices
    # share a 32-bit word with the operation kind and flag bits, so the highest rows of both
    # tables are hit on purpose (MVCC's version words and GPUTx's state words span them too).
    n0 = (1 << 28) - 16
    tabs = [np.arange(n0, dtype=np.int64).reshape(n0, 1), np.arange(32, dtype=np.int64).reshape(16, 2)]
    rng = np.random.Generator(np.random.PCG64(90))
    lengths, row, table, field, kind, arg = [], [], [], [], [], []
    for _ in range(3_000):
        picks = set()
        while len(picks) < 4:
            picks.add((0, n0 - 1 - int(rng.integers(0, 600))) if rng.random() < 0.7 else (1, int(rng.integers(0, 16))))
        for t_, r_ in sorted(picks):
            row.append(r_); table.append(t_); field.append(int(rng.integers(0, 2)) if t_ == 1 else 0)
            k = int(rng.integers(0, 2)); kind.append(k); arg.append(int(rng.integers(-9, 10)) if k else 0)
        lengths.append(4)
    b = wl._pack(lengths, np.array(row, np.uint32), np.array(table, np.uint16), np.array(field, np.uint8),
                 np.array(kind, np.uint8), np.array(arg, np.int64), {})
    print(f"[gpu] maximum total rows {scheme}", flush=True)
    out, reads, final, st = run_batch(tabs, b, scheme)
    assert "error" not in st, st["error"]
    assert np.all(out["status"] == oracle.COMMITTED)
    if scheme in ("gacco", "gputx"):
        exp_fin, exp_reads = oracle.id_order_expected(tabs, b)
        assert np.array_equal(np.asarray(reads, np.int64), exp_reads)
        assert all(np.array_equal(g, x) for g, x in zip(final, exp_fin))
    else:
        assert check(tabs, b, out, reads, final).ok
    # the rows no transaction touched still hold their initial values (spot check of the low end)
    assert np.array_equal(final[0][:1000, 0], np.arange(1000))


@pytest.mark.parametrize("scheme", IMPLEMENTED)
def test_strict_fences(scheme):
    b_ = binding()
    tabs, b = wl.kv_workload(n_rows=20_000, n_fields=4, n_txns=20_000, ops=16, theta=0.99, seed=7)
    run_and_check(tabs, b, scheme, flags=b_.CC_RUN_STRICT_FENCES)


@pytest.mark.skip(reason="CC_RUN_WAIT_UNLOCK is switched off: two teams of one wavefront that block each other "
                         "see the row free on the next loop iteration and retry in lockstep, which livelocked "
                         "the final single-wavefront pass (a GPU run went silent); cc_run rejects the flag")
@pytest.mark.parametrize("scheme", IMPLEMENTED)
def test_wait_unlock_retry_policy(scheme):
    b_ = binding()
    tabs, b = wl.kv_workload(n_rows=20_000, n_fields=4, n_txns=20_000, ops=16, theta=0.99, seed=27)
    run_and_check(tabs, b, scheme, flags=b_.CC_RUN_WAIT_UNLOCK)
    tabs, b = wl.order_entry_workload(1, 1_000, seed=28)
    run_and_check(tabs, b, scheme, flags=b_.CC_RUN_WAIT_UNLOCK)


def test_wait_unlock_flag_is_rejected():
    b_ = binding()
    tabs, b = wl.kv_workload(n_rows=1_000, n_fields=2, n_txns=100, ops=4, seed=29)
    with b_.Engine(tabs) as eng:
        bid = eng.submit(b, "occ")
        with pytest.raises(b_.CCError) as e:
            eng.run(bid, flags=b_.CC_RUN_WAIT_UNLOCK)
        assert e.value.status == b_.CC_E_INVAL
        assert np.array_equal(eng.tables()[0], tabs[0])


@pytest.mark.parametrize("shape", [(16, 1), (64, 1), (4, 2), (1, 1), (1, 4)])
@pytest.mark.parametrize("scheme", ["occ", "tictoc"])
def test_wait_for_blocking_row(scheme, shape):
    # CC_RUN_WAIT_BLOCKER: a failed attempt waits (bounded) for the row another transaction held,
    # in passes that defer; the final pass backs off (the team-loop CPU model's rule)
    b_ = binding()
    lanes, waves = shape
    print(f"[gpu] wait-for-blocker {scheme} L={lanes} waves={waves}", flush=True)
    tabs, b = wl.kv_workload(n_rows=20_000, n_fields=4, n_txns=20_000, ops=(1, 16) if lanes == 1 else 16,
                             theta=0.99, seed=47)
    f = b_.CC_RUN_WAIT_BLOCKER | (b_.CC_RUN_NO_HOT_ENGINE if scheme == "occ" else 0)
    _, _, _, st = run_and_check(tabs, b, scheme, flags=f, lanes_per_txn=lanes, waves_per_wg=waves)
    assert st["blocked_waits"] > 0
    # every transaction adds to both of two rows: the pairs that block each other
    b2 = wl.kv_batch(2, 1, 5_000, ops=2, read_ratio=0.3, arg_range=(-5, 5), seed=48)
    run_and_check([wl.kv_table(2, 1)], b2, scheme, flags=f, lanes_per_txn=max(lanes, 4), waves_per_wg=waves)
    if lanes >= 16:
        tabs, b = wl.order_entry_workload(1, 1_000, seed=49)
        run_and_check(tabs, b, scheme, flags=f, lanes_per_txn=64, waves_per_wg=waves)


@pytest.mark.parametrize("pre", [0, 1, 2])
def test_wait_for_blocking_row_with_each_precheck_setting(pre):
    b_ = binding()
    f = b_.CC_RUN_WAIT_BLOCKER | [b_.CC_RUN_NO_PRECHECK, 0, b_.CC_RUN_PRECHECK][pre] | b_.CC_RUN_NO_HOT_ENGINE
    tabs, b = wl.kv_workload(n_rows=50_000, n_fields=4, n_txns=30_000, ops=16, theta=0.9, seed=50 + pre)
    run_and_check(tabs, b, "occ", flags=f)
    run_and_check(tabs, b, "occ", flags=f | b_.CC_RUN_STRICT_FENCES)


@pytest.mark.parametrize("flags", ["precheck", "precheck+eager", "no-precheck", "precheck+latch"])
@pytest.mark.parametrize("theta", [0.6, 0.99])
@pytest.mark.parametrize("scheme", ["occ", "to", "mvcc", "tictoc"])
def test_precheck(scheme, theta, flags):
    # the pre-check round on every attempt, never, or (default) on retries of a contended batch
    b_ = binding()
    if flags == "precheck+eager" and scheme != "occ":
        pytest.skip("eager install is an OCC option")
    f = {"precheck": b_.CC_RUN_PRECHECK, "precheck+eager": b_.CC_RUN_PRECHECK | b_.CC_RUN_EAGER_INSTALL,
         "no-precheck": b_.CC_RUN_NO_PRECHECK, "precheck+latch": b_.CC_RUN_PRECHECK | b_.CC_RUN_LATCH}[flags]
    if scheme == "occ":
        f |= b_.CC_RUN_NO_HOT_ENGINE  # the rounds of the transaction kernel (the engine has no pre-check)
    tabs, b = wl.kv_workload(n_rows=20_000, n_fields=4, n_txns=20_000, ops=16, theta=theta, seed=37)
    run_and_check(tabs, b, scheme, flags=f)
    tabs, b = wl.order_entry_workload(1, 1_000, seed=38)
    run_and_check(tabs, b, scheme, flags=f)


@pytest.mark.parametrize("pre", ["default", "precheck", "no-precheck"])
@pytest.mark.parametrize("hot", ["hot-last", "one-round"])
@pytest.mark.parametrize("shape", [(16, 1), (64, 1), (4, 2), (1, 1)])
def test_occ_hot_rows_last(shape, hot, pre):
    # the batch's hottest rows locked in a round of their own after every other row; each
    # acquisition of the most written row that does not fail commits exactly one write to it
    b_ = binding()
    f = {"hot-last": b_.CC_RUN_HOT_LAST, "one-round": b_.CC_RUN_NO_HOT_LAST}[hot]
    f |= {"default": 0, "precheck": b_.CC_RUN_PRECHECK, "no-precheck": b_.CC_RUN_NO_PRECHECK}[pre]
    f |= b_.CC_RUN_NO_HOT_ENGINE
    lanes, waves = shape
    if lanes == 1 and hot == "hot-last":
        pytest.skip("the split lock rounds faulted the GPU in the 1-lane, 16-slot kernel with no cause found in "
                    "the source; they are compiled out of the 1-lane and 16-slot variants and this case stays off "
                    "the GPU")
    tabs, b = wl.kv_workload(n_rows=20_000, n_fields=4, n_txns=20_000, ops=16, theta=0.99, seed=41)
    _, _, _, st = run_and_check(tabs, b, "occ", flags=f, lanes_per_txn=lanes, waves_per_wg=waves)
    # one table, distinct rows per transaction: the most written row's write ops are its write accesses
    h = wl.hottest_row_writes(b)[1]
    assert st["hot_writes"] == h
    assert st["hot_acq"] - st["hot_failed"] == h
    assert st["hot_hold_ns"] > 0
    # order-entry at one warehouse (its row written by every payment; slots, conditional adds)
    tabs, b = wl.order_entry_workload(1, 1_500, seed=42)
    # (new-orders reach 66 ops: one 64-lane team per transaction)
    _, _, fin, st = run_and_check(tabs, b, "occ", flags=f, lanes_per_txn=64, waves_per_wg=waves)
    assert oracle.order_entry_invariants(tabs, fin, b, np.ones(b.n_txns, bool)) == []
    assert st["hot_acq"] - st["hot_failed"] == st["hot_writes"]


@pytest.mark.parametrize("theta", [0.6, 0.99])
def test_occ_eager_install(theta):
    # values stored in the validation round and undone on abort; aborted
    # attempts release with a fresh TID
    b_ = binding()
    f = b_.CC_RUN_EAGER_INSTALL | b_.CC_RUN_NO_HOT_ENGINE
    tabs, b = wl.kv_workload(n_rows=20_000, n_fields=4, n_txns=20_000, ops=16, theta=theta, seed=17)
    run_and_check(tabs, b, "occ", flags=f)
    tabs, b = wl.order_entry_workload(1, 1_000, seed=18)
    run_and_check(tabs, b, "occ", flags=f)


@pytest.mark.parametrize("scheme", IMPLEMENTED)
def test_repeated_runs_accumulate(scheme):
    tabs, b = wl.kv_workload(n_rows=10_000, n_fields=2, n_txns=8_000, ops=8, theta=0.9, seed=8)
    bb = binding()
    with bb.Engine(tabs) as eng:
        bid = eng.submit(b, scheme)
        cur = tabs
        for _ in range(3):
            eng.run(bid)
            out, reads = eng.outcomes(bid, b.n_txns, b.total_ops)
            final = eng.tables()
            rep = check(cur, b, out, reads, final)
            assert rep.ok, rep
            cur = final


@pytest.mark.parametrize("scheme", IMPLEMENTED)
def test_attempt_limit_reports_livelock_and_leaves_no_partial_writes(scheme):
    bb = binding()
    n = 4_000
    b = wl.kv_batch(2, 1, n, ops=2, read_ratio=0.0, seed=9)
    tabs = [wl.kv_table(2, 1)]
    # (OCC without the hot-row engine, where conflicts on the two rows wait instead of aborting)
    f = bb.CC_RUN_NO_HOT_ENGINE if scheme == "occ" else 0
    out, reads, final, st = run_batch(tabs, b, scheme, max_attempts=1, lanes_per_txn=4, flags=f)
    assert isinstance(st.get("error"), bb.CCError) and st["error"].status == bb.CC_E_LIVELOCK
    committed = out["status"] == 1
    assert 0 < committed.sum() < n
    # the committed subset is serializable and the aborted ones left nothing behind
    rep = check(tabs, b, out, reads, final, require_all_committed=False)
    assert rep.ok, rep
    assert np.all(out["attempts"][~committed] == 1)


@pytest.mark.parametrize("scheme", IMPLEMENTED)
def test_full_size_kv_config(scheme):
    # the headline configuration: 10M rows x 10 fields, 1M transactions x 16 ops, Zipf 0.9
    tabs, b = wl.kv_workload(theta=0.9, seed=0)
    out, reads, final, st = run_and_check(tabs, b, scheme)
    print(f"full {scheme}: {b.n_txns / (st['run_ns'] * 1e-9):.3e} txn/s attempts={st['attempts']}")


def test_full_size_kv_config_without_hot_engine():
    # the headline configuration through OCC's transaction kernel alone
    b_ = binding()
    tabs, b = wl.kv_workload(theta=0.9, seed=0)
    _, _, _, st = run_and_check(tabs, b, "occ", flags=b_.CC_RUN_NO_HOT_ENGINE)
    assert st["engine_txns"] == 0


def test_hot_engine_plan_follows_its_rule():
    # the engine rows: the most written rows (most first, ties by row), at most 32, each written at
    # least max(2, n_txns / 4096) times; its transactions: those that write one of them
    b_ = binding()
    tabs, b = wl.kv_workload(theta=0.9, seed=0)
    with b_.Engine(tabs) as eng:
        bid = eng.submit(b, "occ")
        rows, n_eng, by_default = b_.cc_engine_plan(eng.ctx, bid)
        bid2 = eng.submit(b, "tictoc")
        assert b_.cc_engine_plan(eng.ctx, bid2)[1] == 0  # OCC only
    w = b.kind != wl.READ
    cnt = np.bincount(b.row[w].astype(np.int64), minlength=len(tabs[0]))
    thr = max(2, b.n_txns // 4096)
    order = np.lexsort((np.arange(len(cnt)), -cnt))
    exp = [int(r) for r in order[:32] if cnt[r] >= thr]
    assert rows.tolist() == exp
    txn_of_op = np.repeat(np.arange(b.n_txns), b.n_ops.astype(np.int64))
    hit = np.zeros(b.n_txns, bool)
    hit[txn_of_op[w & np.isin(b.row, exp)]] = True
    assert n_eng == int(hit.sum())
    # used by default: the most written row left out is written at most a quarter as often as the first
    assert by_default == bool(cnt[order[len(exp)]] * 4 <= cnt[order[0]])


def test_full_size_kv_config_runs_the_hot_engine_by_default():
    tabs, b = wl.kv_workload(theta=0.9, seed=0)
    _, _, _, st = run_and_check(tabs, b, "occ")
    h = wl.hottest_row_writes(b)[1]
    print(f"engine: {st['engine_txns']} txns, {st['engine_rows']} rows, {st['engine_ns'] / 1e6:.1f} ms of "
          f"{st['run_ns'] / 1e6:.1f} ms; hot row {h} writes, {st['hot_acq']} holds")
    assert st["engine_txns"] > 0 and st["engine_rows"] == 32
    assert st["hot_acq"] - st["hot_failed"] == h


@pytest.mark.parametrize("theta", [0.6, 0.9, 0.99])
@pytest.mark.parametrize("shape", [(16, 0), (16, 1), (64, 0), (4, 0), (4, 2), (1, 0)])
def test_hot_engine(shape, theta):
    # the transactions that write the batch's most written rows run first in one workgroup that
    # holds those rows in LDS (waiting for them, the most written last); the rest run as usual
    b_ = binding()
    lanes, waves = shape
    print(f"[gpu] hot engine L={lanes} waves={waves} theta={theta}", flush=True)
    tabs, b = wl.kv_workload(n_rows=20_000, n_fields=4, n_txns=20_000, ops=(1, 4) if lanes == 1 else 16,
                             theta=theta, seed=61)
    _, _, _, st = run_and_check(tabs, b, "occ", flags=b_.CC_RUN_HOT_ENGINE, lanes_per_txn=lanes, waves_per_wg=waves)
    assert st["engine_txns"] > 0 and 0 < st["engine_rows"] <= 32
    # every write of the most written row happens in the engine, one per held lock that committed
    h = wl.hottest_row_writes(b)[1]
    assert st["hot_acq"] - st["hot_failed"] == h
    assert st["hot_hold_ns"] > 0
    # the same with strict fences
    run_and_check(tabs, b, "occ", flags=b_.CC_RUN_HOT_ENGINE | b_.CC_RUN_STRICT_FENCES, lanes_per_txn=lanes,
                  waves_per_wg=waves)


@pytest.mark.parametrize("waves", [0, 1, 4])
def test_hot_engine_order_entry_and_tiny_tables(waves):
    b_ = binding()
    # order-entry at one and eight warehouses: slots, conditional adds, several ops per row
    for w in (1, 8):
        print(f"[gpu] hot engine order-entry W={w} waves={waves}", flush=True)
        tabs, b = wl.order_entry_workload(w, 2_000, seed=62 + w)
        _, _, fin, st = run_and_check(tabs, b, "occ", flags=b_.CC_RUN_HOT_ENGINE, lanes_per_txn=64,
                                      waves_per_wg=waves)
        assert oracle.order_entry_invariants(tabs, fin, b, np.ones(b.n_txns, bool)) == []
        assert st["engine_txns"] > 0
    # every transaction writes both rows of a two-row table: the whole batch runs in the engine
    print(f"[gpu] hot engine two rows waves={waves}", flush=True)
    b2 = wl.kv_batch(2, 1, 5_000, ops=2, read_ratio=0.3, arg_range=(-5, 5), seed=63)
    _, _, _, st = run_and_check([wl.kv_table(2, 1)], b2, "occ", flags=b_.CC_RUN_HOT_ENGINE, lanes_per_txn=4,
                                waves_per_wg=waves)
    writes = sum(1 for t in range(b2.n_txns) if (b2.kind[b2.txn_slice(t)] != wl.READ).any())
    assert st["engine_txns"] == writes
    # a tiny batch
    tabs, b = wl.tiny_workload(seed=64)
    run_and_check(tabs, b, "occ", flags=b_.CC_RUN_HOT_ENGINE, waves_per_wg=waves)


def test_hot_engine_needs_at_most_four_ops_per_lane():
    b_ = binding()
    tabs, b = wl.kv_workload(n_rows=20_000, n_fields=4, n_txns=2_000, ops=16, theta=0.9, seed=65)
    with b_.Engine(tabs) as eng:
        bid = eng.submit(b, "occ")
        with pytest.raises(b_.CCError) as e:
            eng.run(bid, flags=b_.CC_RUN_HOT_ENGINE, lanes_per_txn=1)
        assert e.value.status == b_.CC_E_INVAL
        # the refused run left the batch as it was: it runs afterwards
        eng.run(bid, flags=b_.CC_RUN_HOT_ENGINE, lanes_per_txn=16)
        out, reads = eng.outcomes(bid, b.n_txns, b.total_ops)
        assert check(tabs, b, out, reads, eng.tables()).ok
    # by default the engine is simply not used there
    _, _, _, st = run_and_check(tabs, b, "occ", lanes_per_txn=1)
    assert st["engine_txns"] == 0


@pytest.mark.parametrize("scheme", IMPLEMENTED)
@pytest.mark.parametrize("warehouses", [1, 8])
def test_order_entry(scheme, warehouses):
    # multi-table transactions with conditional adds, cross-row slot writes and several
    # field operations per row; W=1 puts every payment on one warehouse row
    tabs, b = wl.order_entry_workload(warehouses, 1_500, seed=warehouses)
    out, reads, final, st = run_and_check(tabs, b, scheme)
    assert oracle.order_entry_invariants(tabs, final, b, out["status"] == 1) == []


@functools.lru_cache(maxsize=1)
def _order_entry_64():
    # the order-entry configuration at its largest size: 64 warehouses (6.4M stock rows, 1.92M customers)
    return wl.order_entry_workload(64, 20_000, seed=64)


@pytest.mark.parametrize("scheme", IMPLEMENTED + ["gacco", "gputx"])
def test_order_entry_64_warehouses(scheme):
    tabs, b = _order_entry_64()
    print(f"[gpu] order-entry W=64 {scheme}: {b.n_txns} txns, {b.total_ops} ops", flush=True)
    out, reads, final, st = run_batch(tabs, b, scheme)
    assert "error" not in st, st["error"]
    assert np.all(out["status"] == oracle.COMMITTED)
    if scheme in ("gacco", "gputx"):
        exp_fin, exp_reads = oracle.id_order_expected(tabs, b)
        assert np.array_equal(np.asarray(reads, np.int64), exp_reads)
        assert all(np.array_equal(g, x) for g, x in zip(final, exp_fin))
    rep = check(tabs, b, out, reads, final)
    assert rep.ok, rep
    assert oracle.order_entry_invariants(tabs, final, b, out["status"] == 1) == []


@pytest.mark.parametrize("scheme", ["to", "mvcc"])
def test_timestamp_overflow_is_reported(scheme):
    bb = binding()
    tabs, b = wl.kv_workload(n_rows=1_000, n_fields=2, n_txns=5_000, ops=4, theta=0.9, seed=10)
    out, reads, final, st = run_batch(tabs, b, scheme, ts_start=(1 << 31) - 2_000)
    assert isinstance(st.get("error"), bb.CCError) and st["error"].status == bb.CC_E_TS_OVERFLOW
    # what did commit is still a serializable prefix, and nothing else was written
    rep = check(tabs, b, out, reads, final, require_all_committed=False)
    assert rep.ok, rep
    assert (out["status"] == 1).sum() < b.n_txns


@pytest.mark.parametrize("scheme", ["occ", "tictoc", "2pl_nw"])
def test_large_ticket_start_is_harmless(scheme):
    tabs, b = wl.kv_workload(n_rows=1_000, n_fields=2, n_txns=5_000, ops=4, theta=0.9, seed=10)
    run_and_check(tabs, b, scheme, ts_start=(1 << 40))


# ---------------------------------------------------------------------------
# epoch mode (batching): graph-replayed epochs, aborted transactions retried in
# the next epoch
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("scheme", IMPLEMENTED)
def test_epoch_mode(scheme):
    bb = binding()
    tabs, b = wl.kv_workload(n_rows=100_000, n_fields=4, n_txns=20_000, ops=(2, 64), theta=0.8, seed=21)
    out, reads, final, st = run_and_check(tabs, b, scheme, mode=bb.CC_MODE_EPOCH)
    assert st["epochs"] >= 4 and st["epochs"] % 4 == 0


@functools.lru_cache(maxsize=1)
def _uneven_full():
    # the batching configuration at its largest batch: 2^20 transactions of 2-64 ops, Zipf 0.8,
    # on the 10M-row x 10-field table
    return wl.kv_workload(n_txns=1 << 20, ops=(2, 64), theta=0.8, seed=0)


@pytest.mark.parametrize("scheme", ["occ", "tictoc"])
def test_epoch_mode_full_batch(scheme):
    bb = binding()
    tabs, b = _uneven_full()
    print(f"[gpu] epoch mode, 2^20 uneven txns ({b.total_ops} ops), {scheme}", flush=True)
    out, reads, final, st = run_and_check(tabs, b, scheme, mode=bb.CC_MODE_EPOCH)
    assert st["epochs"] >= 4
    assert np.array_equal(final[0], oracle.final_add_only(tabs, b)[0])
    print(f"[gpu] epochs={st['epochs']} passes={st['passes']} {b.n_txns / (st['run_ns'] * 1e-9):.3e} txn/s", flush=True)


@pytest.mark.parametrize("scheme", ["occ", "tictoc"])
def test_epoch_graph_replays(scheme):
    # the captured graph is reused by later runs of the batch; every replay must
    # be valid and end in the order-free closed form
    bb = binding()
    tabs, b = wl.kv_workload(n_rows=50_000, n_fields=4, n_txns=12_000, ops=(2, 32), theta=0.9, seed=22)
    cf = oracle.final_add_only(tabs, b)
    with bb.Engine(tabs) as eng:
        bid = eng.submit(b, scheme)
        for rep in range(4):
            eng.load(tabs)
            st = eng.run(bid, mode=bb.CC_MODE_EPOCH, lanes_per_txn=16)
            out, reads = eng.outcomes(bid, b.n_txns, b.total_ops)
            final = eng.tables()
            r = check(tabs, b, out, reads, final)
            assert r.ok, (rep, r)
            assert np.array_equal(final[0], cf[0])
            # a plain run in between must not disturb the cached graph
            if rep == 1:
                eng.load(tabs)
                eng.run(bid)


@pytest.mark.parametrize("scheme", ["occ", "2pl_nw"])
def test_epoch_limit_reports_livelock(scheme):
    bb = binding()
    b = wl.kv_batch(2, 1, 3_000, ops=2, read_ratio=0.0, seed=23)
    tabs = [wl.kv_table(2, 1)]
    out, reads, final, st = run_batch(tabs, b, scheme, mode=bb.CC_MODE_EPOCH, max_epochs=4)
    assert isinstance(st.get("error"), bb.CCError) and st["error"].status == bb.CC_E_LIVELOCK
    assert check(tabs, b, out, reads, final, require_all_committed=False).ok


def test_autotuner_picks_a_feasible_point():
    bb = binding()
    from paper_2406_10158_amd import autotune
    tabs, b = wl.kv_workload(n_rows=100_000, n_fields=4, n_txns=16_384, ops=(2, 64), theta=0.8, seed=24)
    with bb.Engine(tabs) as eng:
        bid = eng.submit(b, "occ")
        best, res = autotune.tune(eng, bid, b.n_txns, reset=lambda: eng.load(tabs))
        assert best is not None and best["feasible"]
        infeasible = [r for r in res if not r["feasible"]]
        assert any(r["lanes_per_txn"] == 1 for r in infeasible)  # 64-op transactions do not fit one lane
        # the chosen point still produces a correct run
        eng.load(tabs)
        params = {k: best[k] for k in ("mode", "lanes_per_txn", "waves_per_wg", "grid", "defer_after")}
        eng.run(bid, **params)
        out, reads = eng.outcomes(bid, b.n_txns, b.total_ops)
        assert check(tabs, b, out, reads, eng.tables()).ok


# ---------------------------------------------------------------------------
# Latch variants (CC_RUN_LATCH): every control-word update becomes a critical
# section under a per-row 32-bit latch; the outcome must still be serializable.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme", IMPLEMENTED)
@pytest.mark.parametrize("theta", [0.6, 0.99])
def test_latch_variants_kv(scheme, theta):
    b_ = binding()
    tabs, b = wl.kv_workload(n_rows=20_000, n_fields=4, n_txns=20_000, ops=16, theta=theta, seed=41)
    run_and_check(tabs, b, scheme, flags=b_.CC_RUN_LATCH)


@pytest.mark.parametrize("scheme", IMPLEMENTED)
def test_latch_variants_hot_rows_order_entry_and_tiny(scheme):
    b_ = binding()
    n = 20_000
    b = wl.kv_batch(2, 1, n, ops=2, read_ratio=0.3, arg_range=(-5, 5), seed=42)
    run_and_check([wl.kv_table(2, 1)], b, scheme, lanes_per_txn=4, flags=b_.CC_RUN_LATCH)
    tabs, b = wl.order_entry_workload(1, 1_000, seed=43)
    run_and_check(tabs, b, scheme, flags=b_.CC_RUN_LATCH | b_.CC_RUN_STRICT_FENCES)
    for seed in range(4):
        tabs, b = wl.kv_workload(n_rows=3, n_fields=1, n_txns=7, ops=(1, 3), theta=0.0, seed=200 + seed)
        out, reads, final, st = run_batch(tabs, b, scheme, lanes_per_txn=1, waves_per_wg=1, flags=b_.CC_RUN_LATCH)
        assert "error" not in st
        assert oracle.bruteforce_count(tabs, b, np.arange(b.n_txns), reads, final) >= 1


def test_latch_variant_in_epoch_mode():
    b_ = binding()
    tabs, b = wl.kv_workload(n_rows=20_000, n_fields=4, n_txns=20_000, ops=(2, 64), theta=0.8, seed=44)
    run_and_check(tabs, b, "occ", mode=b_.CC_MODE_EPOCH, lanes_per_txn=64, flags=b_.CC_RUN_LATCH)
