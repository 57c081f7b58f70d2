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
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the engine is single-device (no multi-GPU path is built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2406_10158_amd import binding, workload

    t_gen = time.time()
    tables, batch = workload.kv_workload(n_rows=args.rows, n_fields=args.fields, n_txns=args.txns, ops=args.ops,
                                         theta=args.theta, seed=args.seed)
    t_gen = time.time() - t_gen
    print(f"[bench] generated {batch.n_txns} txns / {batch.total_ops} ops in {t_gen:.1f}s", file=sys.stderr,
          flush=True)
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    eng = binding.Engine(tables, device=0, stream=stream.cuda_stream)
    bid = eng.submit(batch, args.scheme)
    params = dict(lanes_per_txn=args.lanes, waves_per_wg=args.waves, grid=args.grid, flags=args.flags)
    for _ in range(args.warmup):
        eng.run(bid, **params)
    torch.cuda.synchronize()
    kernel_ns, run_ns, attempts, p50, p99 = [], [], [], [], []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = eng.run(bid, **params)
        kernel_ns.append(st["kernel_ns"])
        run_ns.append(st["run_ns"])
        attempts.append(st["attempts"])
        p50.append(st["lat_p50_ns"])
        p99.append(st["lat_p99_ns"])
        print(f"[bench] step: {st['run_ns'] / 1e6:.2f} ms, attempts {st['attempts']}", file=sys.stderr, flush=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    ms_per_step = ms_total / args.steps
    value = batch.n_txns / (ms_per_step / 1e3)

    alg = algorithmic_bytes(batch)
    k_s = float(np.mean(kernel_ns)) * 1e-9
    achieved = alg / k_s / 1e9
    traffic = None
    if os.path.exists(args.traffic_json):
        with open(args.traffic_json) as f:
            tj = json.load(f)
        key = f"{args.scheme}:{args.theta}:{args.rows}x{args.fields}:{args.txns}x{args.ops}"
        traffic = tj.get(key)
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": "txn_kernel", "algorithmic_bytes_per_launch": alg,
                "kernel_ms": round(k_s * 1e3, 3)}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        oracle.serial_execute(tables, batch)
        dt = time.perf_counter() - t
        cpu = {"value": round(batch.n_txns / dt, 1), "unit": "txn/s", "cores": 1, "kind": "oracle",
               "sample": f"serial execution (oracle_replay in id order) of all {batch.n_txns} transactions of "
                         f"the same batch, {dt:.2f} s on one host core"}

    wl_name = (f"kv {args.rows} rows x {args.fields} int64 fields, {args.txns} txns x {args.ops} ops, "
               f"read ratio 0.5, zipf {args.theta}, {args.scheme}")
    res = {
        "metric": METRIC, "value": round(value, 1), "unit": "txn/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": wl_name, "rows": args.rows, "fields": args.fields, "txns": args.txns,
                   "ops_per_txn": args.ops, "theta": args.theta, "read_ratio": 0.5, "scheme": args.scheme,
                   "lanes_per_txn": args.lanes, "waves_per_wg": args.waves, "grid": args.grid,
                   "global_batch": args.txns, "parallelism": "single GPU"},
        "p50_commit_latency_ms": round(float(np.median(p50)) / 1e6, 4),
        "p99_commit_latency_ms": round(float(np.median(p99)) / 1e6, 4),
        "abort_rate": round((float(np.mean(attempts)) - batch.n_txns) / batch.n_txns, 4),
        "kernel_only_txn_per_s": round(batch.n_txns / k_s, 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "host_wall_s": round(wall, 3),
    }
    eng.close()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
