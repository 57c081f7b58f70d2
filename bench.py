"""Benchmark: committed transactions per second of the HIP engine on one MI355X.

One step = one cc_run of the whole hot path on one resident batch: CC
initialisation (control words reset) plus the transaction kernel that runs
every transaction to commit.  Default workload: key-value table of 10M rows x
10 int64 fields, 1M transactions x 16 ops (read ratio 0.5, RMW adds U[-100,100]),
Zipf 0.9 keys, OCC.  Inputs are synthetic (seeded generator).

Prints one JSON line.  Usage:
  python bench.py [--steps K] [--warmup W] [--scheme occ] [--theta 0.9]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "committed txns/sec on 1 MI355X (Zipf 0.9 KV, 16 ops/txn) + p99 commit latency"
HBM_PEAK_GBS = 8000.0


# the sources a kernel's HBM counters depend on (profiles/traffic.json keys them by their hash)
KERNEL_SOURCES = {"txn_kernel": ("kernels.hip", "schemes.h", "txn_kernel.h", "device.h"),
                  "engine_kernel": ("hot_engine.h", "schemes.h", "device.h")}


def algorithmic_bytes(batch) -> int:
    """Bytes the OCC hot path must move for one committed pass over the batch.

    Per op: its 16 B descriptor and its 8 B read value out, plus the 8 B value
    read; per row access (row-group leader): the 8 B control word touched once
    (lock or load); per written op: the 8 B value stored; per written row: the
    8 B word store that releases it; per read-only row: the 8 B validation
    re-load.  Per transaction: the 8 B descriptor and the 32 B outcome.
    """
    kind = batch.kind
    n_ops = batch.total_ops
    # row groups: an op starts a group unless it repeats the previous op's (table,row) in its txn
    first = np.zeros(n_ops, bool)
    first[batch.first_op[batch.n_ops > 0].astype(np.int64)] = True
    same = np.zeros(n_ops, bool)
    same[1:] = (batch.row[1:] == batch.row[:-1]) & (batch.table[1:] == batch.table[:-1])
    leader = first | ~same
    grp = np.cumsum(leader) - 1
    written_grp = np.zeros(int(leader.sum()), bool)
    np.logical_or.at(written_grp, grp, kind != 0)
    n_groups = len(written_grp)
    n_wgroups = int(written_grp.sum())
    n_writes = int((kind != 0).sum())
    return (n_ops * (16 + 8 + 8) + n_groups * 8 + n_writes * 8 + n_wgroups * 8 + (n_groups - n_wgroups) * 8
            + batch.n_txns * (8 + 32))


def access_counts(batch) -> dict:
    """Memory operations one committed pass of the OCC hot path must issue, from the batch itself.

    Control words (8 B per row, 80 MB for 10M rows) and values (the 800 MB
    value arena) are separate arrays, so their random accesses are counted
    apart: they are priced at the rates of their own footprints.
    """
    kind = batch.kind
    n_ops = batch.total_ops
    first = np.zeros(n_ops, bool)
    first[batch.first_op[batch.n_ops > 0].astype(np.int64)] = True
    same = np.zeros(n_ops, bool)
    same[1:] = (batch.row[1:] == batch.row[:-1]) & (batch.table[1:] == batch.table[:-1])
    leader = first | ~same
    grp = np.cumsum(leader) - 1
    written = np.zeros(int(leader.sum()), bool)
    np.logical_or.at(written, grp, kind != 0)
    n_groups, n_wgroups = len(written), int(written.sum())
    n_writes = int((kind != 0).sum())
    return {
        "value_loads": n_ops,                          # every op reads its value
        "word_loads": 2 * (n_groups - n_wgroups),      # read-only rows: word + validation re-read
        "word_atomics": n_wgroups,                     # write-row try-locks
        "value_stores": n_writes,                      # new values
        "word_stores": n_wgroups,                      # publishing words
        "stream_bytes": n_ops * (16 + 8) + batch.n_txns * (8 + 32),
    }


def run_probes(ctx, binding, batch=None, quick=False) -> dict:
    """Self-measured rates of the memory operations the hot path is made of.

    Random 8-byte coherent loads at three footprints: 80 MB (the 10M-row
    control-word array, which fits the 256 MB Infinity Cache), 880 MB (words
    plus the 800 MB value arena) and 1.4 GB; stores at 80 and 880 MB; 64-bit
    fetch_or at 80 MB with uniform addresses and, given a batch, at the
    batch's own written rows (its Zipf distribution, in batch order); the
    single-word hand-off and the OCC commit hand-off with the second side on
    the same CU, on another CU of the same XCD, and on another XCD.
    """
    n_cu, _ = binding.cc_device_info(ctx)
    threads = n_cu * 8 * 256

    def ops_of(n):
        per = ((n + threads - 1) // threads + 3) // 4 * 4
        return threads * per

    out = {}
    n = 1 << (26 if quick else 28)
    ms = binding.cc_probe(ctx, "stream", 2 << 30, 0)
    out["stream_GBps"] = ((2 << 30) // 32 * 32) / ms / 1e6  # half the buffer read, half written
    for mb in (80, 880, 1400):
        out[f"gather_{mb}MB_Gops"] = ops_of(n) / binding.cc_probe(ctx, "gather", mb * 1_000_000, n) / 1e6
    for mb in (80, 880):
        out[f"scatter_{mb}MB_Gops"] = ops_of(n) / binding.cc_probe(ctx, "scatter", mb * 1_000_000, n) / 1e6
    out["atomic_80MB_Gops"] = ops_of(n) / binding.cc_probe(ctx, "atomic", 80_000_000, n) / 1e6
    if batch is not None:
        rows = batch.row[batch.kind != 0].astype(np.uint64)
        if len(rows):
            ms = binding.cc_probe_indices(ctx, "atomic", max(80_000_000, (int(rows.max()) + 4) * 8), rows)
            out["atomic_batch_rows_Gops"] = len(rows) / ms / 1e6
    rounds = 4000 if quick else 20000
    for name, peer in (("same_cu", 0), ("same_xcd", 8), ("cross_xcd", 1)):
        ms = binding.cc_probe(ctx, "handoff", 1 << 20, rounds, peer)
        out[f"handoff_{name}_ns"] = ms * 1e6 / (2 * rounds)
        ms = binding.cc_probe(ctx, "commit_handoff", 1 << 20, rounds, peer)
        out[f"commit_handoff_{name}_ns"] = ms * 1e6 / rounds
    # the hot row is touched from every XCD: the bounds take the cross-XCD hand-offs
    out["handoff_ns"] = out["handoff_cross_xcd_ns"]
    out["commit_handoff_ns"] = out["commit_handoff_cross_xcd_ns"]
    # OCC's hot-row engine passes its rows between wavefronts of one workgroup, in LDS
    out["engine_handoff_ns"] = binding.cc_probe(ctx, "engine_handoff", 1 << 20, rounds) * 1e6 / rounds
    ms = binding.cc_probe(ctx, "wave_counter", 1 << 20, 1 << 26)
    out["one_word_atomic_ns"] = ms * 1e6 / (threads // 64 * (((1 << 26) + threads - 1) // threads + 3) // 4 * 4)
    return {k: round(v, 3) for k, v in out.items()}



def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(tables, batch, out, reads, final) -> dict:
    """The oracle timed on this host's cores, on the same batch the GPU ran.

    Leg 1, serial replay: the whole batch executed one transaction at a time
    in id order (one core), repeated on fresh table copies until ~10 s have
    been timed.  Leg 2, per-key checker: the GPU run's outcome (serial keys,
    every read value, the final table) checked cell by cell on every core the
    process may use (C + OpenMP), repeated until ~10 s have been timed.
    """
    import oracle
    model = _cpu_model()
    host_cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    reps, dt = 0, 0.0
    while reps == 0 or dt < 10.0:
        t = time.perf_counter()
        oracle.serial_execute(tables, batch)
        dt += time.perf_counter() - t
        reps += 1
    serial = {"name": "serial replay", "value": round(reps * batch.n_txns / dt, 1), "unit": "txn/s", "cores": 1,
              "cpu_model": model,
              "sample": f"all {batch.n_txns} transactions of the batch executed in id order, {reps} times, "
                        f"{dt:.1f} s on one core"}
    preps, pdt, threads, ok = 0, 0.0, 0, True
    while preps == 0 or pdt < 10.0:
        t = time.perf_counter()
        rep = oracle.check_run_perkey(tables, batch, out["status"], out["serial_hi"], out["serial_lo"], reads, final,
                                      threads=0)
        pdt += time.perf_counter() - t
        preps += 1
        threads, ok = rep.threads, ok and rep.ok
    perkey = {"name": "per-key checker", "value": round(preps * batch.n_txns / pdt, 1), "unit": "txn/s checked",
              "cores": int(threads), "host_cores": int(host_cores), "cpu_model": model, "run_ok": bool(ok),
              "sample": f"the GPU run's outcome ({batch.n_txns} transactions, every read value, the final table) "
                        f"checked {preps} times, {pdt:.1f} s on {threads} threads"}
    return {"value": serial["value"], "unit": "txn/s", "cores": 1, "kind": "oracle", "cpu_model": model,
            "sample": serial["sample"], "legs": [serial, perkey]}


def _emit(rec):
    print(json.dumps(rec), flush=True)


def _run_stats(eng, bid, n_txns, steps=2, warmup=1, reset=None, **params):
    for _ in range(warmup):
        if reset:
            reset()
        eng.run(bid, **params)
    sts = []
    for _ in range(steps):
        if reset:
            reset()
        sts.append(eng.run(bid, **params))
    run_ns = float(np.median([s["run_ns"] for s in sts]))
    st = sts[-1]
    att = float(np.mean([s["attempts"] for s in sts]))
    busy = st["t_useful_ns"] + st["t_abort_ns"] + st["t_wait_ns"]
    return {"txn_per_s": round(n_txns / (run_ns * 1e-9), 1), "run_ms": round(run_ns / 1e6, 3),
            "kernel_ms": round(st["kernel_ns"] / 1e6, 3), "abort_rate": round((att - n_txns) / max(n_txns, 1), 3),
            "p50_ms": round(st["lat_p50_ns"] / 1e6, 4), "p99_ms": round(st["lat_p99_ns"] / 1e6, 4),
            "passes": st["passes"], "epochs": st["epochs"],
            "breakdown": {k: round(st[f"t_{k}_ns"] / busy, 3) if busy else 0 for k in ("useful", "abort", "wait")}}


def _pick(args, names):
    """The suite's schemes, narrowed to --only when it is given."""
    only = [x for x in (args.only or "").split(",") if x]
    return tuple(n for n in names if not only or n in only)


def suite_schemes(args, binding, workload):
    """Every scheme on the key-value config at each contention level."""
    for theta in (0.0, 0.6, 0.9, 0.99):
        tables, batch = workload.kv_workload(n_rows=args.rows, n_fields=args.fields, n_txns=args.txns,
                                             ops=args.ops, theta=theta, seed=args.seed)
        h = workload.hottest_row_writes(batch)[1]
        # the oracle beside the GPU: its serial replay of the same batch on one host core
        import oracle
        t0 = time.perf_counter()
        oracle.serial_execute(tables, batch)
        dt = time.perf_counter() - t0
        _emit({"suite": "schemes", "theta": theta, "scheme": "oracle (serial replay, 1 host core)",
               "txn_per_s": round(batch.n_txns / dt, 1), "run_ms": round(dt * 1e3, 3)})
        eng = binding.Engine(tables)
        for scheme in _pick(args, ("occ", "2pl_nw", "2pl_wd", "to", "mvcc", "tictoc", "gacco", "gputx")):
            bid = eng.submit(batch, scheme)
            rec = {"suite": "schemes", "theta": theta, "scheme": scheme, "hot_row_writes": h}
            try:
                rec.update(_run_stats(eng, bid, batch.n_txns))
                if scheme == "gputx":
                    rec["ksets"] = binding.cc_stats(eng.ctx, bid)["ksets"]
            except binding.CCError as e:
                rec["error"] = str(e)
            _emit(rec)
            eng.release(bid)
        eng.close()


def suite_order_entry(args, binding, workload):
    """Order-entry (NewOrder + Payment) at 1, 8 and 64 warehouses under every scheme."""
    import oracle
    for w in (1, 8, 64):
        tables, batch = workload.order_entry_workload(w, args.oe_txns, seed=args.seed)
        eng = binding.Engine(tables)
        for scheme in _pick(args, ("occ", "2pl_nw", "2pl_wd", "to", "mvcc", "tictoc", "gacco", "gputx")):
            bid = eng.submit(batch, scheme)
            rec = {"suite": "order_entry", "warehouses": w, "txns": batch.n_txns, "scheme": scheme}
            try:
                eng.load(tables)
                rec.update(_run_stats(eng, bid, batch.n_txns, steps=1, warmup=0))
                out, reads = eng.outcomes(bid, batch.n_txns, batch.total_ops)
                fin = eng.tables()
                rep = oracle.check_run(tables, batch, out["status"], out["serial_hi"], out["serial_lo"], reads, fin)
                rec["oracle_ok"] = bool(rep.ok)
                rec["invariants"] = oracle.order_entry_invariants(tables, fin, batch, out["status"] == 1)
            except binding.CCError as e:
                rec["error"] = str(e)
            _emit(rec)
            eng.release(bid)
        eng.close()


def suite_index(args, binding, workload):
    """Key-value batches that name rows by key: no index, binary search, 16-way tree (OCC and GaccO)."""
    keys = workload.index_keys(args.rows, seed=args.seed)
    # the oracle beside the GPU: dictionary resolution of a sample of keys on one host core
    import oracle
    sample = workload.kv_batch(args.rows, args.fields, 20_000, ops=args.ops, theta=0.0, seed=args.seed)
    sample_keys = workload.keyed_ops(sample, [keys])
    t0 = time.perf_counter()
    oracle.resolve_keys([keys], sample, sample_keys)
    dt = time.perf_counter() - t0
    _emit({"suite": "index", "lookup": "oracle (dictionary, 1 host core)", "keys": int(sample.total_ops),
           "seconds": round(dt, 3), "note": "includes building the dictionary of all keys"})
    for theta in (0.0, 0.6, 0.9):
        tables, batch = workload.kv_workload(n_rows=args.rows, n_fields=args.fields, n_txns=args.txns,
                                             ops=args.ops, theta=theta, seed=args.seed)
        op_keys = workload.keyed_ops(batch, [keys])
        eng = binding.Engine(tables)
        eng.create_index(0, keys)
        for scheme in ("occ", "gacco"):
            for method in ("none", "bsearch", "tree"):
                bid = eng.submit(batch, scheme) if method == "none" else eng.submit_keyed(batch, op_keys, scheme)
                flags = binding.CC_RUN_INDEX_TREE if method == "tree" else 0
                rec = {"suite": "index", "theta": theta, "scheme": scheme, "lookup": method}
                try:
                    rec.update(_run_stats(eng, bid, batch.n_txns, flags=flags))
                    st = binding.cc_stats(eng.ctx, bid)
                    rec["index_ms"] = round(st["index_ns"] / 1e6, 3)
                    rec["index_share"] = round(st["index_ns"] / max(st["run_ns"], 1), 3)
                except binding.CCError as e:
                    rec["error"] = str(e)
                _emit(rec)
                eng.release(bid)
        eng.close()


def suite_latch(args, binding, workload):
    """Latch-free (default) against latched control-word updates, every non-deterministic scheme."""
    for theta in (0.0, 0.6, 0.9):
        tables, batch = workload.kv_workload(n_rows=args.rows, n_fields=args.fields, n_txns=args.txns,
                                             ops=args.ops, theta=theta, seed=args.seed)
        eng = binding.Engine(tables)
        for scheme in _pick(args, ("occ", "2pl_nw", "2pl_wd", "to", "mvcc", "tictoc")):
            bid = eng.submit(batch, scheme)
            for latch in (False, True):
                rec = {"suite": "latch", "theta": theta, "scheme": scheme, "latch": latch}
                try:
                    rec.update(_run_stats(eng, bid, batch.n_txns, steps=1, warmup=1,
                                          flags=binding.CC_RUN_LATCH if latch else 0))
                except binding.CCError as e:
                    rec["error"] = str(e)
                _emit(rec)
            eng.release(bid)
        eng.close()


def suite_ycsb(args, binding, workload):
    """The paper's YCSB presets (RO, MC, HC) and its two sweeps (Exp-1: theta at W=0.1; Exp-2: W at theta=0.6)."""
    configs = [("RO", 0.0, 0.0), ("MC", 0.1, 0.6), ("HC", 0.5, 0.8)]
    configs += [("exp1", 0.1, th) for th in (0.0, 0.3, 0.6, 0.8, 0.9)]
    configs += [("exp2", w, 0.6) for w in (0.0, 0.3, 0.5, 0.7, 0.9)]
    variants = [(s_, 0) for s_ in _pick(args, ("occ", "2pl_nw", "2pl_wd", "to", "mvcc", "tictoc", "gacco", "gputx"))]
    if _pick(args, ("gacco+shared_reads",)):
        variants.append(("gacco", binding.CC_RUN_SHARED_READS))
    for name, w, theta in configs:
        tables, batch = workload.kv_workload(n_rows=args.rows, n_fields=args.fields, n_txns=args.txns,
                                             ops=args.ops, read_ratio=1.0 - w, theta=theta, seed=args.seed)
        eng = binding.Engine(tables)
        for scheme, flags in variants:
            bid = eng.submit(batch, scheme)
            rec = {"suite": "ycsb", "set": name, "W": w, "theta": theta,
                   "scheme": scheme + ("+shared_reads" if flags else "")}
            try:
                rec.update(_run_stats(eng, bid, batch.n_txns, steps=1, warmup=1, flags=flags))
            except binding.CCError as e:
                rec["error"] = str(e)
            _emit(rec)
            eng.release(bid)
        eng.close()


def suite_batching(args, binding, workload):
    """Uneven transactions (2-64 ops), Zipf 0.8: autotuned plain and epoch launches per batch size."""
    from paper_2406_10158_amd import autotune
    cache = autotune.TuneCache(os.path.join(ROOT, "paper_2406_10158_amd", "tuned.json"))
    tables, full = workload.kv_workload(n_rows=args.rows, n_fields=args.fields, n_txns=1 << 20, ops=(2, 64),
                                        theta=0.8, seed=args.seed)
    eng = binding.Engine(tables)
    for lg in range(14, 21):
        batch = full if lg == 20 else full.subset(np.arange(1 << lg))
        bid = eng.submit(batch, "occ")
        default = _run_stats(eng, bid, batch.n_txns, steps=1, warmup=1)
        best, res = autotune.tune(eng, bid, batch.n_txns,
                                  log=lambda r: print(f"[tune] {batch.n_txns} {r.get('mode_name')} "
                                                      f"L={r['lanes_per_txn']} W={r['waves_per_wg']} "
                                                      f"{r.get('txn_per_s', 'infeasible')}", file=sys.stderr,
                                                      flush=True))
        key = autotune.TuneCache.key("kv-uneven-2-64", 0.8, batch.n_txns, "occ")
        cache.put(key, best)
        by_mode = {}
        for r in res:
            if r["feasible"]:
                m = r["mode_name"]
                if m not in by_mode or r["txn_per_s"] > by_mode[m]["txn_per_s"]:
                    by_mode[m] = r
        _emit({"suite": "batching", "batch": batch.n_txns, "default_plain": default,
               "best": {m: {k: r[k] for k in ("lanes_per_txn", "waves_per_wg", "defer_after", "txn_per_s", "run_ms",
                                              "attempts", "epochs", "p99_ms")} for m, r in by_mode.items()},
               "infeasible": sum(1 for r in res if not r["feasible"]), "points": len(res)})
        eng.release(bid)
    cache.save()
    eng.close()


def suite_epoch(args, binding, workload):
    """The batching configuration's largest batch (2^20 transactions of 2-64 ops, Zipf 0.8) run once in
    plain mode and once in epoch mode (one warm-up each), for a kernel trace of the epoch graph."""
    tables, batch = workload.kv_workload(n_rows=args.rows, n_fields=args.fields, n_txns=1 << 20, ops=(2, 64),
                                         theta=0.8, seed=args.seed)
    eng = binding.Engine(tables)
    bid = eng.submit(batch, "occ")
    for mode, name in ((binding.CC_MODE_PLAIN, "plain"), (binding.CC_MODE_EPOCH, "epoch")):
        for rep in range(2):
            eng.load(tables)
            st = eng.run(bid, mode=mode)
        _emit({"suite": "epoch", "mode": name, "txns": batch.n_txns, "txn_per_s": round(batch.n_txns / (st["run_ns"] * 1e-9), 1),
               "run_ms": round(st["run_ns"] / 1e6, 3), "kernel_ms": round(st["kernel_ns"] / 1e6, 3),
               "epochs": st["epochs"], "passes": st["passes"], "attempts": st["attempts"]})
    eng.close()


def suite_serving(args, binding, workload):
    """Poisson streams of key-value (8-32 ops, Zipf 0.9) + order-entry (W=8) at increasing offered load.

    One stream of --serve-arrivals transactions is generated once (in parallel
    processes for long streams) and its arrival times are rescaled for each
    offered load, so the 1M txn/s point spans arrivals / 1M seconds.  OCC runs
    every load under the --serve-cap admission budget; MVCC then runs the 2M
    txn/s point with the version arena sized by a 64 MB cap and without a cap,
    to show that the cap bounds the arena whatever the stream's length.
    """
    t0 = time.time()
    workers = min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count() or 1)
    tables, batch, arr1, m = workload.serve_stream(
        args.serve_arrivals, 1e6, kv_rows=args.rows, kv_fields=args.fields, seed=args.seed, workers=workers,
        log=lambda msg: print(f"[serving] {msg} ({time.time() - t0:.0f}s)", file=sys.stderr, flush=True))
    print(f"[serving] {batch.n_txns} arrivals, {batch.total_ops} ops generated in {time.time() - t0:.0f}s "
          f"({workers} processes)", file=sys.stderr, flush=True)
    eng = binding.Engine(tables)

    def point(scheme, rate, cap, bid):
        arr = (arr1 * (1e6 / rate)).astype(np.int64)
        binding.cc_set_arrivals(eng.ctx, bid, arr)
        rec = {"suite": "serving", "scheme": scheme, "offered_txn_per_s": rate, "arrivals": batch.n_txns,
               "stream_span_s": round(float(arr[-1]) / 1e9, 3), "hbm_cap_bytes": cap}
        try:
            eng.load(tables)
            st = eng.run(bid, mode=binding.CC_MODE_SERVE, hbm_cap_bytes=cap)
            out, _ = eng.outcomes(bid, batch.n_txns, 0)
            span_ns = float(out["commit_ns"].max())
            committed_rate = st["committed"] / (span_ns * 1e-9)
            rec.update(committed=st["committed"], committed_txn_per_s=round(committed_rate, 1),
                       p50_latency_ms=round(st["lat_p50_ns"] / 1e6, 4), p99_latency_ms=round(st["lat_p99_ns"] / 1e6, 4),
                       abort_rate=round((st["attempts"] - st["committed"]) / max(st["committed"], 1), 3),
                       admit_waits=st["admit_waits"], passes=st["passes"],
                       # below saturation the engine keeps up with the offered load, the queue stays
                       # short and the latencies are the steady state's; above it they grow with the
                       # backlog, i.e. with the stream's length
                       steady_state=bool(committed_rate >= 0.99 * rate))
            if scheme == "mvcc":
                rec.update(version_slots=st["version_slots"], version_arena_bytes=st["version_slots"] * 32,
                           version_misses=st["version_misses"], writes=int((batch.kind != 0).sum()))
        except binding.CCError as e:
            rec["error"] = str(e)
        _emit(rec)
        print(f"[serving] {scheme} {rate:.0e}: {rec.get('committed_txn_per_s')} txn/s, "
              f"p99 {rec.get('p99_latency_ms')} ms", file=sys.stderr, flush=True)

    bid = eng.submit(batch, "occ")
    for rate in (1e6, 2e6, 5e6, 10e6, 20e6, 50e6):
        point("occ", rate, args.serve_cap, bid)
    eng.release(bid)
    bid = eng.submit(batch, "mvcc")
    for cap in (64 << 20, 0):
        point("mvcc", 2e6, cap, bid)
    eng.release(bid)
    eng.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scheme", default="occ")
    ap.add_argument("--theta", type=float, default=0.9)
    ap.add_argument("--rows", type=int, default=10_000_000)
    ap.add_argument("--fields", type=int, default=10)
    ap.add_argument("--txns", type=int, default=1_000_000)
    ap.add_argument("--ops", type=int, default=16)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--flags", type=int, default=0)
    ap.add_argument("--defer-after", type=int, default=0, help="attempts before a transaction is deferred to the next pass (0: the library default)")
    ap.add_argument("--backoff-ns", type=int, default=0, help="back-off base (OCC family) or poll interval per queued access (GaccO, GPUTx); 0: the library default, 200 ns")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probes", action="store_true", help="only run the memory micro-benchmarks")
    ap.add_argument("--suite", choices=["schemes", "order_entry", "batching", "serving", "index", "latch", "ycsb",
                                        "epoch"],
                    help="run a measurement suite instead of the headline step (JSON line per point)")
    ap.add_argument("--only", default="", help="comma-separated schemes a suite runs (default: all of its schemes)")
    ap.add_argument("--oe-txns", type=int, default=100_000)
    ap.add_argument("--serve-arrivals", type=int, default=100_000)
    ap.add_argument("--serve-cap", type=int, default=4 << 30)
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the engine is single-device (no multi-GPU path is built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2406_10158_amd import binding, workload

    if args.probes:
        ctx = binding.cc_init(0)
        _, b = workload.kv_workload(n_rows=args.rows, n_fields=args.fields, n_txns=args.txns, ops=args.ops,
                                    theta=args.theta, seed=args.seed)
        print(json.dumps({"probes": run_probes(ctx, binding, batch=b)}))
        binding.cc_destroy(ctx)
        return
    if args.suite:
        {"schemes": suite_schemes, "order_entry": suite_order_entry, "batching": suite_batching, "index": suite_index,
         "latch": suite_latch, "ycsb": suite_ycsb, "epoch": suite_epoch,
         "serving": suite_serving}[args.suite](args, binding, workload)
        return

    t_gen = time.time()
    tables, batch = workload.kv_workload(n_rows=args.rows, n_fields=args.fields, n_txns=args.txns, ops=args.ops,
                                         theta=args.theta, seed=args.seed)
    t_gen = time.time() - t_gen
    print(f"[bench] generated {batch.n_txns} txns / {batch.total_ops} ops in {t_gen:.1f}s", file=sys.stderr,
          flush=True)
    torch.cuda.init()
    stream = torch.cuda.Stream()  # default priority; the engine issues all its work on it
    eng = binding.Engine(tables, device=0, stream=stream.cuda_stream)
    bid = eng.submit(batch, args.scheme)
    params = dict(lanes_per_txn=args.lanes, waves_per_wg=args.waves, grid=args.grid, flags=args.flags,
                  defer_after=args.defer_after, backoff_ns=args.backoff_ns)
    # pristine copies of the tables in device memory: every step starts from
    # the same table, restored device-to-device outside the timed region
    pristine = [torch.from_numpy(np.ascontiguousarray(t)).to("cuda") for t in tables]

    def restore():
        with torch.cuda.stream(stream):
            for tid, t in zip(eng.ids, pristine):
                binding.cc_load(eng.ctx, tid, t)

    for _ in range(args.warmup):
        restore()
        eng.run(bid, **params)
    torch.cuda.synchronize()
    kernel_ns, run_ns, attempts, p50, p99, passes, step_ms, engine_ns = [], [], [], [], [], [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        restore()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        st = eng.run(bid, **params)
        ev1.record(stream)
        ev1.synchronize()
        step_ms.append(ev0.elapsed_time(ev1))
        kernel_ns.append(st["kernel_ns"])
        run_ns.append(st["run_ns"])
        attempts.append(st["attempts"])
        p50.append(st["lat_p50_ns"])
        p99.append(st["lat_p99_ns"])
        passes.append(st["passes"])
        engine_ns.append(st["engine_ns"])
        print(f"[bench] step: {step_ms[-1]:.2f} ms, attempts {st['attempts']}, passes {st['passes']}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = float(np.median(step_ms))
    value = batch.n_txns / (ms_per_step / 1e3)
    # the last step ran once from the pristine tables: its outcome is what the CPU checker times
    out_last, reads_last = eng.outcomes(bid, batch.n_txns, batch.total_ops)
    final_last = eng.tables()

    # HBM roofline of the dominant kernel (algorithmic bytes / its time): the
    # transaction kernel, or, when OCC's hot-row engine ran, the engine over
    # its own share of the batch
    eng_rows, _, _ = binding.cc_engine_plan(eng.ctx, bid) if args.scheme == "occ" else (np.zeros(0), 0, False)
    eng_txns = np.zeros(0, np.int64)
    if len(engine_ns) and np.mean(engine_ns) > 0:
        w = batch.kind != workload.READ
        txn_of_op = np.repeat(np.arange(batch.n_txns), batch.n_ops.astype(np.int64))
        hit = np.zeros(batch.n_txns, bool)
        hit[txn_of_op[w & (batch.table == 0) & np.isin(batch.row, eng_rows)]] = True
        eng_txns = np.nonzero(hit)[0]
    k_step_s = float(np.mean(kernel_ns)) * 1e-9
    if len(eng_txns):
        alg = algorithmic_bytes(batch.subset(eng_txns))
        dom_s, launches, dom_kernel = float(np.mean(engine_ns)) * 1e-9, 1.0, "engine_kernel"
    else:
        alg = algorithmic_bytes(batch)
        dom_s, launches = k_step_s, float(np.mean(passes))
        dom_kernel = {"gacco": "gacco_kernel", "gputx": "gputx_exec_kernel"}.get(args.scheme, "txn_kernel")
    achieved = alg / dom_s / 1e9
    traffic = None
    if os.path.exists(args.traffic_json):
        import hashlib
        with open(args.traffic_json) as f:
            tj = json.load(f)
        t = tj.get(f"{args.scheme}:{args.theta}:{args.rows}x{args.fields}:{args.txns}x{args.ops}:{dom_kernel}")
        csrc = os.path.join(ROOT, "paper_2406_10158_amd", "csrc")
        cur = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read()
                                      for f in KERNEL_SOURCES.get(dom_kernel, KERNEL_SOURCES["txn_kernel"]))).hexdigest()[:16]
        # counters taken on another version of the kernel do not describe this one
        if t and t.get("kernel_src_sha256_16") == cur:
            traffic = t["total_bytes_per_launch"]
    roofline = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic,
                "kernel": dom_kernel,
                "launches_per_step": launches,
                "algorithmic_bytes_per_launch": int(alg / launches),
                "avg_launch_ms": round(dom_s * 1e3 / launches, 4)}

    # measured random-access / atomic roofline and hot-row contention bound
    probes = run_probes(eng.ctx, binding, batch=batch, quick=True)
    acc = access_counts(batch)
    # control words at the 80 MB rates, values at the 880 MB rates
    t_roof = (acc["word_loads"] / (probes["gather_80MB_Gops"] * 1e9)
              + acc["value_loads"] / (probes["gather_880MB_Gops"] * 1e9)
              + acc["word_atomics"] / (probes["atomic_80MB_Gops"] * 1e9)
              + acc["value_stores"] / (probes["scatter_880MB_Gops"] * 1e9)
              + acc["word_stores"] / (probes["scatter_80MB_Gops"] * 1e9)
              + acc["stream_bytes"] / (probes["stream_GBps"] * 1e9))
    x_roof = batch.n_txns / t_roof
    if args.scheme == "gacco":
        # every access of the hottest row (reads too) is one turn of its word;
        # the bound takes the plain store-to-load hand-off per turn
        _, h = workload.hottest_row_accesses(batch)
        t_h, h_key = probes["handoff_ns"], "hot_row_accesses_H"
    elif args.scheme == "gputx":
        # the rank pass hands the hottest row along its accesses, one turn
        # each; then the K-sets run one after another, each released by the
        # done counter: at least one store-to-load hand-off per turn and per K-set
        _, h = workload.hottest_row_accesses(batch)
        h += int(st["ksets"])
        t_h, h_key = probes["handoff_ns"], "hot_row_accesses_plus_ksets_H"
    else:
        _, h = workload.hottest_row_writes(batch)
        t_h, h_key = probes["commit_handoff_ns"], "hot_row_writes_H"
    x_cont = batch.n_txns / (h * t_h * 1e-9) if h else float("inf")
    engine_bound = None
    if len(eng_txns):
        # the engine runs before the rest of the batch: the passes' bounds add.
        # Engine: its hottest row's writes at the engine's hand-off; rest: its
        # own hottest row at OCC's commit hand-off, or its random accesses.
        rest = batch.subset(np.setdiff1d(np.arange(batch.n_txns), eng_txns))
        _, h_rest = workload.hottest_row_writes(rest)
        acc_r = access_counts(rest)
        t_rest_roof = (acc_r["word_loads"] / (probes["gather_80MB_Gops"] * 1e9)
                       + acc_r["value_loads"] / (probes["gather_880MB_Gops"] * 1e9)
                       + acc_r["word_atomics"] / (probes["atomic_80MB_Gops"] * 1e9)
                       + acc_r["value_stores"] / (probes["scatter_880MB_Gops"] * 1e9)
                       + acc_r["word_stores"] / (probes["scatter_80MB_Gops"] * 1e9)
                       + acc_r["stream_bytes"] / (probes["stream_GBps"] * 1e9))
        t_eng = h * probes["engine_handoff_ns"] * 1e-9
        t_rest = max(h_rest * probes["commit_handoff_ns"] * 1e-9, t_rest_roof)
        x_cont = batch.n_txns / (t_eng + t_rest)
        engine_bound = {"engine_txns": int(len(eng_txns)), "engine_rows": int(len(eng_rows)),
                        "t_h_engine_ns": probes["engine_handoff_ns"], "engine_min_ms": round(t_eng * 1e3, 3),
                        "rest_hot_row_writes": int(h_rest), "rest_min_ms": round(t_rest * 1e3, 3),
                        "engine_ms": round(float(np.mean(engine_ns)) / 1e6, 3)}
    eff = min(x_roof, x_cont)
    measured = {"random_access_roof_txn_per_s": round(x_roof, 1), h_key: h,
                "t_h_ns": t_h, "contention_bound_txn_per_s": round(x_cont, 1),
                "effective_roof_txn_per_s": round(eff, 1), "active_bound": "contention" if x_cont < x_roof else "random-access",
                "frac_of_effective": round(value / eff, 4), "hot_row_engine": engine_bound, "probes": probes,
                "per_batch_accesses": acc}

    roofline["active_bound"] = measured["active_bound"]
    roofline["active"] = {"achieved": round(value, 1), "peak": round(eff, 1), "unit": "txn/s",
                          "frac": round(value / eff, 4),
                          "peak_from": ("hot-row engine, then the rest of the batch: H x the engine's LDS hand-off, "
                                        "plus the rest's hottest row x the commit hand-off (or its random accesses)"
                                        if engine_bound and measured["active_bound"] == "contention" else
                                        "H x t_h: writes to the hottest row times the measured commit hand-off"
                                        if measured["active_bound"] == "contention" else
                                        "random loads, atomics, stores and streamed bytes at the probed rates")}

    # the batch's most written row during the last step (OCC's lock-hold counters)
    hot_row = None
    if args.scheme == "occ" and st["hot_acq"]:
        # with the engine, the row is written only while the engine runs
        span = st["engine_ns"] if st["engine_txns"] else st["kernel_ns"]
        held = st["hot_hold_ns"] / max(span, 1)
        hot_row = {"writes_H": st["hot_writes"], "lock_acquisitions": st["hot_acq"],
                   "failed_holds": st["hot_failed"], "held_share": round(held, 4), "idle_share": round(1 - held, 4),
                   "hold_per_acquisition_ns": round(st["hot_hold_ns"] / st["hot_acq"], 1),
                   "kernel_ns_per_hot_commit": round(span / max(st["hot_writes"], 1), 1),
                   "in": "engine_kernel" if st["engine_txns"] else "txn_kernel"}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(tables, batch, out_last, reads_last, final_last)
    wl_name = (f"kv {args.rows} rows x {args.fields} int64 fields, {args.txns} txns x {args.ops} ops, "
               f"read ratio 0.5, zipf {args.theta}, {args.scheme}")
    res = {
        "metric": METRIC, "value": round(value, 1), "unit": "txn/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": wl_name, "rows": args.rows, "fields": args.fields, "txns": args.txns,
                   "ops_per_txn": args.ops, "theta": args.theta, "read_ratio": 0.5, "scheme": args.scheme,
                   "lanes_per_txn": args.lanes, "waves_per_wg": args.waves, "grid": args.grid,
                   "defer_after": args.defer_after, "backoff_ns": args.backoff_ns, "global_batch": args.txns, "parallelism": "single GPU"},
        "p50_commit_latency_ms": round(float(np.median(p50)) / 1e6, 4),
        "p99_commit_latency_ms": round(float(np.median(p99)) / 1e6, 4),
        "abort_rate": round((float(np.mean(attempts)) - batch.n_txns) / batch.n_txns, 4),
        "kernel_only_txn_per_s": round(batch.n_txns / k_step_s, 1),
        "step_ms": {"median": round(ms_per_step, 4), "mean": round(float(np.mean(step_ms)), 4),
                    "min": round(float(np.min(step_ms)), 4), "max": round(float(np.max(step_ms)), 4),
                    "timing": "HIP events around each cc_run on the engine's stream; tables restored "
                              "device-to-device from a pristine copy before each step, outside the events"},
        "roofline": roofline,
        "measured_roofline": measured,
        "hot_row": hot_row,
        "cpu_baseline": cpu,
        "host_wall_s": round(wall, 3),
    }
    eng.close()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
