"""GPU serving mode: continuous admission of a Poisson stream, checked against the oracle.

The alone-versus-mix test runs a key-value stream by itself and interleaved
with an order-entry stream on disjoint tables (same arrival times): every run
must replay exactly in its serial order, the key-value table must end in the
same state (add-only, so it is order-free), and transactions on a reserved
key range nothing else touches must read bit-identical values in both runs.
"""
import numpy as np
import pytest

import oracle
from helpers import SCHEMES, binding, check, run_batch
from paper_2406_10158_amd import workload as wl

pytestmark = pytest.mark.gpu


def serve(tables, batch, arrivals, scheme="occ", **params):
    bb = binding()
    with bb.Engine(tables) as eng:
        bid = eng.submit(batch, scheme)
        bb.cc_set_arrivals(eng.ctx, bid, arrivals)
        err = None
        try:
            st = eng.run(bid, mode=bb.CC_MODE_SERVE, **params)
        except bb.CCError as e:
            err, st = e, bb.cc_stats(eng.ctx, bid)
        out, reads = eng.outcomes(bid, batch.n_txns, batch.total_ops)
        final = eng.tables()
    assert err is None, err
    return out, reads, final, st


@pytest.mark.parametrize("scheme", SCHEMES)
def test_serve_stream_parity(scheme):
    tabs, b, arr, m = wl.serve_stream(6_000, 2e6, kv_rows=200_000, isolated_frac=0.05, seed=31)
    out, reads, final, st = serve(tabs, b, arr, scheme)
    rep = check(tabs, b, out, reads, final)
    assert rep.ok, rep
    # nothing commits before it arrives (device clock ticks are 10 ns)
    assert np.all(out["commit_ns"] + 10 >= arr)
    assert st["lat_p99_ns"] >= st["lat_p50_ns"] > 0


def test_serve_alone_vs_mix():
    kw = dict(kv_rows=200_000, isolated_frac=0.1, seed=32)
    tabs, mix, arr, m = wl.serve_stream(8_000, 4e6, **kw)
    _, alone, arr_a, ma = wl.serve_stream(8_000, 4e6, with_oe=False, **kw)
    out_m, reads_m, fin_m, _ = serve(tabs, mix, arr)
    out_a, reads_a, fin_a, _ = serve(tabs, alone, arr_a)
    assert check(tabs, mix, out_m, reads_m, fin_m).ok
    assert check(tabs, alone, out_a, reads_a, fin_a).ok
    # the key-value table is order-free: same final state alone and in the mix
    cf = oracle.final_add_only([tabs[0]], alone)[0]
    assert np.array_equal(fin_a[0], cf)
    assert np.array_equal(fin_m[0], cf)
    # isolated transactions read the same bytes alone and mixed (their initial values)
    kv_ids_mix = np.nonzero(m["is_kv"])[0]
    iso_a = np.nonzero(ma["is_isolated"])[0]
    assert len(iso_a) > 0
    for t_a in iso_a:
        t_m = kv_ids_mix[t_a]
        ra = reads_a[alone.txn_slice(int(t_a))]
        rm = reads_m[mix.txn_slice(int(t_m))]
        assert np.array_equal(ra, rm)
        sl = alone.txn_slice(int(t_a))
        assert np.array_equal(ra, 16 * alone.row[sl].astype(np.int64) + alone.field[sl].astype(np.int64))


@pytest.mark.parametrize("scheme", ["occ", "mvcc"])
def test_serve_alone_vs_mix_full_size(scheme):
    # the serving configuration's shape: the 10M-row x 10-field key-value table (8-32 ops, Zipf 0.9)
    # mixed 50/50 with order-entry at 8 warehouses, 50k Poisson arrivals at 2M txn/s offered
    kw = dict(kv_rows=10_000_000, isolated_frac=0.05, seed=35)
    tabs, mix, arr, m = wl.serve_stream(50_000, 2e6, **kw)
    _, alone, arr_a, ma = wl.serve_stream(50_000, 2e6, with_oe=False, **kw)
    print(f"[gpu] serving full size {scheme}: mix {mix.n_txns} txns, alone {alone.n_txns}", flush=True)
    out_m, reads_m, fin_m, st_m = serve(tabs, mix, arr, scheme)
    out_a, reads_a, fin_a, st_a = serve(tabs, alone, arr_a, scheme)
    rep = check(tabs, mix, out_m, reads_m, fin_m)
    assert rep.ok, rep
    rep = check(tabs, alone, out_a, reads_a, fin_a)
    assert rep.ok, rep
    assert np.all(out_m["commit_ns"] + 10 >= arr) and np.all(out_a["commit_ns"] + 10 >= arr_a)
    # a served stream never runs OCC's hot-row engine, which knows no arrivals
    assert st_m["engine_txns"] == 0 and st_a["engine_txns"] == 0
    cf = oracle.final_add_only([tabs[0]], alone)[0]
    assert np.array_equal(fin_a[0], cf) and np.array_equal(fin_m[0], cf)
    assert oracle.order_entry_invariants(tabs[1:], fin_m[1:], _oe_part(mix, m), out_m["status"][~m["is_kv"]] == 1) == []
    kv_ids_mix = np.nonzero(m["is_kv"])[0]
    iso_a = np.nonzero(ma["is_isolated"])[0]
    assert len(iso_a) > 1000
    for t_a in iso_a:
        ra = reads_a[alone.txn_slice(int(t_a))]
        rm = reads_m[mix.txn_slice(int(kv_ids_mix[t_a]))]
        assert np.array_equal(ra, rm)
    print(f"[gpu] p50/p99 mix {st_m['lat_p50_ns'] / 1e6:.3f}/{st_m['lat_p99_ns'] / 1e6:.3f} ms, "
          f"alone {st_a['lat_p50_ns'] / 1e6:.3f}/{st_a['lat_p99_ns'] / 1e6:.3f} ms", flush=True)


def _oe_part(mix, m):
    """The order-entry transactions of a mixed stream as a batch over the order-entry tables alone."""
    oe_ids = np.nonzero(~m["is_kv"])[0]
    part = wl.concat_batches([(mix, oe_ids)])
    part.table = (part.table - 1).astype(np.uint16)
    part.meta = {"is_new_order": np.array([bool((part.table[part.txn_slice(i)] == wl.T_ORDER).any())
                                           for i in range(part.n_txns)])}
    return part


@pytest.mark.parametrize("scheme", ["occ", "mvcc"])
def test_serve_small_budget_throttles_but_loses_nothing(scheme):
    bb = binding()
    tabs, b, arr, m = wl.serve_stream(3_000, 20e6, kv_rows=100_000, seed=33)
    cap = 3 * 32 * bb.CC_SERVE_BYTES_PER_OP
    out, reads, final, st = serve(tabs, b, arr, scheme, hbm_cap_bytes=cap)
    assert st["admit_waits"] > 0
    assert st["committed"] == b.n_txns
    assert check(tabs, b, out, reads, final).ok


@pytest.mark.parametrize("kv_rows,slots", [(2_000, 1_024), (2_000, 4_096), (100_000, 4_096)])
def test_serve_mvcc_version_arena_bounded_by_the_cap(kv_rows, slots):
    # the cap sizes MVCC's version arena (cap / 32 slots, at least 1024); a stream that commits
    # many times more writes than the arena holds reuses its slots as a ring, and old-version
    # reads whose slot was reused abort and retry -- the run still equals the serial replay
    bb = binding()
    tabs, b, arr, m = wl.serve_stream(30_000, 5e6, kv_rows=kv_rows, seed=36)
    writes = int((b.kind != 0).sum())
    cap = slots * 32
    out, reads, final, st = serve(tabs, b, arr, "mvcc", hbm_cap_bytes=cap)
    assert st["version_slots"] == slots and writes > 100 * slots
    assert st["committed"] == b.n_txns
    rep = check(tabs, b, out, reads, final)
    assert rep.ok, rep
    assert oracle.order_entry_invariants(tabs[1:], final[1:], _oe_part(b, m), out["status"][~m["is_kv"]] == 1) == []
    print(f"[gpu] mvcc serve kv_rows={kv_rows}: {writes} writes through {st['version_slots']} slots, "
          f"{st['version_misses']} version misses", flush=True)
    # without a cap: one slot per op of the stream
    out, reads, final, st = serve(tabs, b, arr, "mvcc")
    assert st["version_slots"] == max(b.total_ops, 1024)
    assert check(tabs, b, out, reads, final).ok


def test_serve_needs_arrivals():
    bb = binding()
    tabs, b, arr, m = wl.serve_stream(100, 1e6, kv_rows=10_000, seed=34)
    with bb.Engine(tabs) as eng:
        bid = eng.submit(b, "occ")
        with pytest.raises(bb.CCError) as e:
            eng.run(bid, mode=bb.CC_MODE_SERVE)
        assert e.value.status == bb.CC_E_STATE
        with pytest.raises(bb.CCError):
            bb.cc_set_arrivals(eng.ctx, bid, arr[::-1].copy() if len(arr) > 1 else np.array([-1]))


@pytest.mark.parametrize("scheme", ["occ", "tictoc", "2pl_wd"])
def test_serve_stream_with_latched_control_words(scheme):
    # the latch variants under continuous admission
    bb = binding()
    tabs, b, arr, m = wl.serve_stream(4_000, 2e6, kv_rows=100_000, seed=33)
    out, reads, final, st = serve(tabs, b, arr, scheme, flags=bb.CC_RUN_LATCH)
    assert check(tabs, b, out, reads, final).ok
    assert np.all(out["commit_ns"] + 10 >= arr)
